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
#include "kernels.h"

namespace relpic {

constexpr int kSeg = 256;
constexpr int kNumXcd = 8;

template <typename Real>
__device__ __forceinline__ Real ldc(const Real *f, long long row, int col) {
  return col >= 0 ? f[row + col] : Real(0);
}

// Workgroup -> (x1 segment, i2, i3), XCD-contiguous.  Returns false for the
// padding workgroups of the last band.
__device__ __forceinline__ bool tile_of(const Geo &g, int nseg, int &l0, int &i2, int &i3) {
  const long long nb = (long long)nseg * g.n2 * g.n3;
  const long long per = (nb + kNumXcd - 1) / kNumXcd;
  const long long bid = blockIdx.x;
  const long long lin = (bid % kNumXcd) * per + bid / kNumXcd;
  if (lin >= nb) return false;
  const int seg = (int)(lin % nseg);
  const long long r = lin / nseg;
  i2 = (int)(r % g.n2);
  i3 = (int)(r / g.n2);
  l0 = seg * kSeg;
  return true;
}

__host__ __device__ inline unsigned tile_blocks(const Geo &g) {
  const long long nseg = (g.n1 + kSeg - 1) / kSeg;
  const long long nb = nseg * g.n2 * g.n3;
  const long long per = (nb + kNumXcd - 1) / kNumXcd;
  return (unsigned)(per * kNumXcd);
}

// Bout = Bin - curl+ E  (coefficients already carry the time step:
// ax.c[l] = C_l c / dx1, h2 = c / dx2, h3 = c / dx3).
template <typename Real, int DIM, int MM>
__global__ __launch_bounds__(kSeg) void k_curl_e(Geo g, Fields<Real> f, const Real *Bin1, const Real *Bin2,
                                                 const Real *Bin3, Real *Bout1, Real *Bout2, Real *Bout3,
                                                 Axial<Real> ax, Real h2, Real h3) {
  __shared__ Real sE2[kSeg + 2 * kMaxM], sE3[kSeg + 2 * kMaxM];
  int l0, i2, i3;
  if (!tile_of(g, (g.n1 + kSeg - 1) / kSeg, l0, i2, i3)) return;
  const int M = MM > 0 ? MM : ax.M;
  const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
  // stage E2, E3 on window cells [l0 - M + 1, l0 + kSeg + M)
  const int span = kSeg + 2 * M;
  for (int t = threadIdx.x; t < span; t += kSeg) {
    const int col = col_of(g, l0 - M + 1 + t);
    sE2[t] = ldc(f.E2, row, col);
    sE3[t] = ldc(f.E3, row, col);
  }
  __syncthreads();
  const int l1 = l0 + threadIdx.x;
  if (l1 >= g.n1) return;
  const int s1 = col_near(g, l1);
  const long long id = row + s1;
  const int c = threadIdx.x + M - 1;  // LDS index of cell l1
  Real d1E2 = 0, d1E3 = 0;
  auto term = [&](int l) {
    d1E2 += ax.c[l - 1] * (sE2[c + l] - sE2[c - l + 1]);
    d1E3 += ax.c[l - 1] * (sE3[c + l] - sE3[c - l + 1]);
  };
  if (MM > 0) {
#pragma unroll
    for (int l = 1; l <= MM; ++l) term(l);
  } else {
    for (int l = 1; l <= M; ++l) term(l);
  }
  const long long row2p = (long long)g.n1 * (wrap_near(i2 + 1, g.n2) + (long long)g.n2 * i3);
  const Real E1 = f.E1[id], E2 = sE2[c], E3 = sE3[c];
  const Real d2E3 = h2 * (f.E3[row2p + s1] - E3);
  const Real d2E1 = h2 * (f.E1[row2p + s1] - E1);
  Real d3E2 = 0, d3E1 = 0;
  if (DIM == 3) {
    const long long row3p = (long long)g.n1 * (i2 + (long long)g.n2 * wrap_near(i3 + 1, g.n3));
    d3E2 = h3 * (f.E2[row3p + s1] - E2);
    d3E1 = h3 * (f.E1[row3p + s1] - E1);
  }
  Bout1[id] = Bin1[id] - (d2E3 - d3E2);
  Bout2[id] = Bin2[id] - (d3E1 - d1E3);
  Bout3[id] = Bin3[id] - (d1E2 - d2E1);
}

// E += curl- B  (ax.c[l] = C_l dt / dx1; e2 = dt / dx2; e3 = dt / dx3).
template <typename Real, int DIM, int MM>
__global__ __launch_bounds__(kSeg) void k_curl_b(Geo g, Fields<Real> f, Axial<Real> ax, Real e2, Real e3) {
  __shared__ Real sB2[kSeg + 2 * kMaxM], sB3[kSeg + 2 * kMaxM];
  int l0, i2, i3;
  if (!tile_of(g, (g.n1 + kSeg - 1) / kSeg, l0, i2, i3)) return;
  const int M = MM > 0 ? MM : ax.M;
  const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
  // stage B2, B3 on window cells [l0 - M, l0 + kSeg + M)
  const int span = kSeg + 2 * M;
  for (int t = threadIdx.x; t < span; t += kSeg) {
    const int col = col_of(g, l0 - M + t);
    sB2[t] = ldc(f.B2, row, col);
    sB3[t] = ldc(f.B3, row, col);
  }
  __syncthreads();
  const int l1 = l0 + threadIdx.x;
  if (l1 >= g.n1) return;
  const int s1 = col_near(g, l1);
  const long long id = row + s1;
  const int c = threadIdx.x + M;  // LDS index of cell l1
  Real d1B3 = 0, d1B2 = 0;
  auto term = [&](int l) {
    d1B3 += ax.c[l - 1] * (sB3[c + l - 1] - sB3[c - l]);
    d1B2 += ax.c[l - 1] * (sB2[c + l - 1] - sB2[c - l]);
  };
  if (MM > 0) {
#pragma unroll
    for (int l = 1; l <= MM; ++l) term(l);
  } else {
    for (int l = 1; l <= M; ++l) term(l);
  }
  const long long row2m = (long long)g.n1 * (wrap_near(i2 - 1, g.n2) + (long long)g.n2 * i3);
  const Real B1 = f.B1[id], B2 = sB2[c], B3 = sB3[c];
  const Real d2B3 = e2 * (B3 - f.B3[row2m + s1]);
  const Real d2B1 = e2 * (B1 - f.B1[row2m + s1]);
  Real d3B2 = 0, d3B1 = 0;
  if (DIM == 3) {
    const long long row3m = (long long)g.n1 * (i2 + (long long)g.n2 * wrap_near(i3 - 1, g.n3));
    d3B2 = e3 * (B2 - f.B2[row3m + s1]);
    d3B1 = e3 * (B1 - f.B1[row3m + s1]);
  }
  f.E1[id] += d2B3 - d3B2;
  f.E2[id] += d3B1 - d1B3;
  f.E3[id] += d1B2 - d2B1;
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
  const JBox b = *box;
  if (b.hi[0] < b.lo[0]) return;
  int lo1 = b.lo[0] - pad, hi1 = b.hi[0] + pad;
  if (g.window) {
    lo1 = lo1 < 0 ? 0 : lo1;
    hi1 = hi1 > g.n1 - 1 ? g.n1 - 1 : hi1;
  } else if (hi1 - lo1 + 1 >= g.n1) {
    lo1 = 0;
    hi1 = g.n1 - 1;
  }
  const long long w1 = hi1 - lo1 + 1, w2 = b.hi[1] - b.lo[1] + 1, w3 = b.hi[2] - b.lo[2] + 1;
  const long long tot = w1 * w2 * w3;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    const int a = (int)(t % w1);
    const long long r = t / w1;
    const int i2 = b.lo[1] + (int)(r % w2);
    const int i3 = b.lo[2] + (int)(r / w2);
    const int col = col_of(g, lo1 + a);
    const long long id = (long long)g.n1 * (i2 + (long long)g.n2 * i3) + col;
    f.E1[id] -= dt * J1src[id];
    f.E2[id] -= dt * f.J2[id];
    f.E3[id] -= dt * f.J3[id];
    f.J1[id] = Real(0);
    f.J2[id] = Real(0);
    f.J3[id] = Real(0);
  }
}

// J1c = G * J1 along x1 inside the current box (x1 widened by ng): FIR with
// taps g_0..g_ng (even in m), zero outside the window or wrapped on a
// periodic line.
template <typename Real>
__global__ __launch_bounds__(256) void k_jcorr(Geo g, const Real *J1, Real *J1c, const Real *taps, int ng,
                                               const JBox *box) {
  const JBox b = *box;
  if (b.hi[0] < b.lo[0]) return;
  int lo1 = b.lo[0] - ng, hi1 = b.hi[0] + ng;
  if (g.window) {
    lo1 = lo1 < 0 ? 0 : lo1;
    hi1 = hi1 > g.n1 - 1 ? g.n1 - 1 : hi1;
  } else if (hi1 - lo1 + 1 >= g.n1) {
    lo1 = 0;
    hi1 = g.n1 - 1;
  }
  const long long w1 = hi1 - lo1 + 1, w2 = b.hi[1] - b.lo[1] + 1, w3 = b.hi[2] - b.lo[2] + 1;
  const long long tot = w1 * w2 * w3;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot; t += (long long)gridDim.x * blockDim.x) {
    const int l1 = lo1 + (int)(t % w1);
    const long long r = t / w1;
    const int i2 = b.lo[1] + (int)(r % w2);
    const int i3 = b.lo[2] + (int)(r / w2);
    const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
    Real acc = taps[0] * ldc(J1, row, col_of(g, l1));
    for (int m = 1; m <= ng; ++m) acc += taps[m] * (ldc(J1, row, col_of(g, l1 - m)) + ldc(J1, row, col_of(g, l1 + m)));
    J1c[row + col_of(g, l1)] = acc;
  }
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
