// Maxwell field advance on the Yee lattice (Eq. 1 with the operators of
// Eq. 14 and, along x1, the customized 2M-point operator of App. C), and the
// J1 current correction of the customized solver (Sec. 3).
//
// B is kept at half-integer times in two buffers, so one step is
//   B^{n+1/2} = B^{n-1/2} - dt d+ x E^n                   (k_curl_e)
//   E^{n+1}   = E^n + dt d- x B^{n+1/2}                    (k_curl_b)
//   E^{n+1}  -= dt J^{n+1/2} inside the deposit's box       (k_add_j)
// which is the leapfrog of the split B half steps; the gather takes
// B^n = (B^{n-1/2} + B^{n+1/2}) / 2.  Each launch maps one workgroup to a
// 256-cell segment of one x1 row; the row and its 2M-cell halo are staged
// in LDS for the axial stencil, and workgroups are renumbered so that each
// XCD sweeps a contiguous band of rows (neighbouring rows share its L2).
#include "field_tiles.h"

namespace relpic {

template <typename Real, int DIM, int MM>
__global__ __launch_bounds__(kSeg) void k_curl_e(Geo g, Fields<Real> f, const Real *Bin1, const Real *Bin2,
                                                 const Real *Bin3, Real *Bout1, Real *Bout2, Real *Bout3,
                                                 Axial<Real> ax, Real h2, Real h3) {
  __shared__ Real sE2[stage_pitch<kSeg>()], sE3[stage_pitch<kSeg>()];
  int l0, i2, i3;
  if (!tile_of(g, (g.n1 + kSeg - 1) / kSeg, l0, i2, i3)) return;
  curl_e_tile<Real, DIM, MM, kSeg, 1>(g, f.E1, f.E2, f.E3, Bin1, Bin2, Bin3, Bout1, Bout2, Bout3, ax, h2, h3, l0, i2, i3,
                                   sE2, sE3);
}

template <typename Real, int DIM, int MM>
__global__ __launch_bounds__(kSeg) void k_curl_b(Geo g, Fields<Real> f, Axial<Real> ax, Real e2, Real e3) {
  __shared__ Real sB2[stage_pitch<kSeg>()], sB3[stage_pitch<kSeg>()];
  int l0, i2, i3;
  if (!tile_of(g, (g.n1 + kSeg - 1) / kSeg, l0, i2, i3)) return;
  curl_b_tile<Real, DIM, MM, kSeg, 1>(g, f.E1, f.E2, f.E3, f.B1, f.B2, f.B3, ax, e2, e3, l0, i2, i3, sB2, sB3);
}

// E -= dt J over the box of deposited current (x1 widened by `pad` for the
// J1 correction's spread), J cleared there; one thread resets the box used
// by the next step's deposit.
template <typename Real>
__global__ __launch_bounds__(256) void k_add_j(Geo g, Fields<Real> f, const Real *J1src, Real dt, const JBox *box,
                                               int pad, JBox *next) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) {
      next->lo[d] = 0x7fffffff;
      next->hi[d] = -0x7fffffff;
    }
  }
  add_j_box(g, f.E1, f.E2, f.E3, f.J1, f.J2, f.J3, J1src, dt, *box, pad,
            blockIdx.x * (long long)blockDim.x + threadIdx.x, (long long)gridDim.x * blockDim.x);
}

// J1c = G * J1 along x1 inside the current box (x1 widened by ng): FIR with
// taps g_0..g_ng (even in m), zero outside the window or wrapped on a
// periodic line.
template <typename Real>
__global__ __launch_bounds__(256) void k_jcorr(Geo g, const Real *J1, Real *J1c, const Real *taps, int ng,
                                               const JBox *box) {
  jcorr_box(g, J1, J1c, taps, ng, *box, blockIdx.x * (long long)blockDim.x + threadIdx.x,
            (long long)gridDim.x * blockDim.x);
}

// Window shift after step n, with g the geometry before the shift.  The
// step's second B half step, B^{n+1} = B^{n+1/2} - (dt/2) curl+ E^{n+1}, is
// taken on the old window, and the window then moves: the back slab (window
// cell 0, storage column `col`) leaves and the same column comes back as the
// new front slab with E^{n+1} = 0 and B^{n+1} = 0.  B is stored at n + 1/2
// and the next step applies the full curl to the shifted E, so two local
// terms keep the result identical:
//   - cells 1..M-1 behind the leaving slab saw its E through the axial
//     stencil during that half step: B^{n+1/2} takes -(dt/2) of the leaving
//     slab's part of curl+ E;
//   - the new front slab gets B^{n+1/2} = (dt/2) curl+ E^{n+1}, whose only
//     terms are the axial ones reaching back into the window.
// ax: C_l (dt/2) / dx1.  The other B buffer's column is cleared.
template <typename Real>
__global__ void k_new_slab(Geo g, Fields<Real> f, Real *Bx1, Real *Bx2, Real *Bx3, int col, Axial<Real> ax) {
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long rows = (long long)g.n2 * g.n3;
  if (r >= rows) return;
  const long long row = r * g.n1;
  const long long id = row + col;
  const Real e2b = f.E2[id], e3b = f.E3[id];
  // old window cells j = 1..M-1 reach the leaving cell 0 through C_{j+1}
  for (int j = 1; j < ax.M; ++j) {
    const long long k = row + col_of(g, j);
    f.B2[k] -= ax.c[j] * e3b;
    f.B3[k] += ax.c[j] * e2b;
  }
  f.E1[id] = f.E2[id] = f.E3[id] = Real(0);
  // new front cell = old window cell n1: d+ f = sum_l C_l (f(n1 + l) - f(n1 - l + 1)),
  // with f zero at old cells >= n1
  Real d1E2 = 0, d1E3 = 0;
  for (int l = 2; l <= ax.M; ++l) {
    const long long k = row + col_of(g, g.n1 - l + 1);
    d1E2 -= ax.c[l - 1] * f.E2[k];
    d1E3 -= ax.c[l - 1] * f.E3[k];
  }
  f.B1[id] = Real(0);
  f.B2[id] = -d1E3;
  f.B3[id] = d1E2;
  Bx1[id] = Bx2[id] = Bx3[id] = Real(0);
}

__global__ void k_reset_box(JBox *b) {
  const int d = threadIdx.x;
  if (d < 3) {
    b->lo[d] = 0x7fffffff;
    b->hi[d] = -0x7fffffff;
  }
}

// ---- launchers ---------------------------------------------------------------

template <typename Real, int DIM>
static void curl_e_dispatch(const Geo &g, const Fields<Real> &f, Real *const Bin[3], Real *const Bout[3],
                            const Axial<Real> &ax, Real h2, Real h3, hipStream_t st) {
  const unsigned nb = tile_blocks(g);
  if (ax.M == 1)
    k_curl_e<Real, DIM, 1><<<nb, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, h3);
  else if (ax.M == 16)
    k_curl_e<Real, DIM, 16><<<nb, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, h3);
  else
    k_curl_e<Real, DIM, 0><<<nb, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, h3);
}

template <typename Real, int DIM>
static void curl_b_dispatch(const Geo &g, const Fields<Real> &f, const Axial<Real> &ax, Real e2, Real e3,
                            hipStream_t st) {
  const unsigned nb = tile_blocks(g);
  if (ax.M == 1)
    k_curl_b<Real, DIM, 1><<<nb, kSeg, 0, st>>>(g, f, ax, e2, e3);
  else if (ax.M == 16)
    k_curl_b<Real, DIM, 16><<<nb, kSeg, 0, st>>>(g, f, ax, e2, e3);
  else
    k_curl_b<Real, DIM, 0><<<nb, kSeg, 0, st>>>(g, f, ax, e2, e3);
}

template <typename Real>
void launch_curl_e(int ndim, const Geo &g, const Fields<Real> &f, Real *const Bin[3], Real *const Bout[3],
                   const Axial<Real> &ax, Real h2, Real h3, hipStream_t st) {
  if (ndim == 3)
    curl_e_dispatch<Real, 3>(g, f, Bin, Bout, ax, h2, h3, st);
  else
    curl_e_dispatch<Real, 2>(g, f, Bin, Bout, ax, h2, h3, st);
}

template <typename Real>
void launch_curl_b(int ndim, const Geo &g, const Fields<Real> &f, const Axial<Real> &ax, Real e2, Real e3,
                   hipStream_t st) {
  if (ndim == 3)
    curl_b_dispatch<Real, 3>(g, f, ax, e2, e3, st);
  else
    curl_b_dispatch<Real, 2>(g, f, ax, e2, e3, st);
}

template <typename Real>
void launch_add_j(const Geo &g, const Fields<Real> &f, const Real *J1src, Real dt, const JBox *box, int pad,
                  JBox *next, hipStream_t st) {
  k_add_j<Real><<<1024, 256, 0, st>>>(g, f, J1src, dt, box, pad, next);
}

template <typename Real>
void launch_jcorr(const Geo &g, const Real *J1, Real *J1c, const Real *taps, int ng, const JBox *box,
                  hipStream_t st) {
  k_jcorr<Real><<<1024, 256, 0, st>>>(g, J1, J1c, taps, ng, box);
}

template <typename Real>
void launch_new_slab(const Geo &g, const Fields<Real> &f, Real *const Bx[3], int col, const Axial<Real> &ax,
                     hipStream_t st) {
  const long long rows = (long long)g.n2 * g.n3;
  k_new_slab<Real><<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(g, f, Bx[0], Bx[1], Bx[2], col, ax);
}

void launch_reset_box(JBox *b, hipStream_t st) { k_reset_box<<<1, 64, 0, st>>>(b); }

#define RELPIC_INST_FIELD(Real)                                                                                   \
  template void launch_curl_e<Real>(int, const Geo &, const Fields<Real> &, Real *const[3], Real *const[3],       \
                                    const Axial<Real> &, Real, Real, hipStream_t);                                \
  template void launch_curl_b<Real>(int, const Geo &, const Fields<Real> &, const Axial<Real> &, Real, Real,      \
                                    hipStream_t);                                                                 \
  template void launch_add_j<Real>(const Geo &, const Fields<Real> &, const Real *, Real, const JBox *, int,     \
                                   JBox *, hipStream_t);                                                          \
  template void launch_jcorr<Real>(const Geo &, const Real *, Real *, const Real *, int, const JBox *,            \
                                   hipStream_t);                                                                  \
  template void launch_new_slab<Real>(const Geo &, const Fields<Real> &, Real *const[3], int, const Axial<Real> &, \
                                      hipStream_t);

RELPIC_INST_FIELD(float)
RELPIC_INST_FIELD(double)

}  // namespace relpic
