// Maxwell field advance on the Yee lattice (Eq. 1 with the operators of
// Eq. 14 and, along x1, the customized 2M-point operator of App. C), and the
// J1 current correction of the customized solver (Sec. 3).
//
// One step of the field phase is  B -= (dt/2) d+ x E ;  E += dt (d- x B - J) ;
// B -= (dt/2) d+ x E  (leapfrog; the two half steps give B at integer times
// for the gather).  All kernels map one thread to one cell, x1 fastest, so
// every load and store is coalesced along x1; neighbours along x1 are shared
// through the L1/LDS path, x2/x3 neighbours are other rows of the same wave's
// footprint and hit L2.
#include "kernels.h"

namespace relpic {

template <typename Real>
__device__ __forceinline__ Real ld(const Real *f, long long row, int col) {
  return col >= 0 ? f[row + col] : Real(0);
}

// B -= h curl+ E.  ax.c[l] = C_l h / dx1; h2 = h / dx2; h3 = h / dx3.
template <typename Real, int DIM, int MM>
__global__ __launch_bounds__(256) void k_bhalf(Geo g, Fields<Real> f, Axial<Real> ax, Real h2, Real h3) {
  const int l1 = blockIdx.x * blockDim.x + threadIdx.x;
  if (l1 >= g.n1) return;
  const int i2 = blockIdx.y, i3 = blockIdx.z;
  const int s1 = col_of(g, l1);
  const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
  const long long id = row + s1;
  const long long row2p = (long long)g.n1 * (wrap(i2 + 1, g.n2) + (long long)g.n2 * i3);
  const int M = MM > 0 ? MM : ax.M;

  Real d1E2 = 0, d1E3 = 0;
  auto term = [&](int l) {
    const int a = col_of(g, l1 + l), b = col_of(g, l1 - l + 1);
    d1E2 += ax.c[l - 1] * (ld(f.E2, row, a) - ld(f.E2, row, b));
    d1E3 += ax.c[l - 1] * (ld(f.E3, row, a) - ld(f.E3, row, b));
  };
  if (MM > 0) {
#pragma unroll
    for (int l = 1; l <= MM; ++l) term(l);
  } else {
    for (int l = 1; l <= M; ++l) term(l);
  }
  const Real E1 = f.E1[id], E2 = f.E2[id], E3 = f.E3[id];
  const Real d2E3 = h2 * (f.E3[row2p + s1] - E3);
  const Real d2E1 = h2 * (f.E1[row2p + s1] - E1);
  Real d3E2 = 0, d3E1 = 0;
  if (DIM == 3) {
    const long long row3p = (long long)g.n1 * (i2 + (long long)g.n2 * wrap(i3 + 1, g.n3));
    d3E2 = h3 * (f.E2[row3p + s1] - E2);
    d3E1 = h3 * (f.E1[row3p + s1] - E1);
  }
  f.B1[id] -= d2E3 - d3E2;
  f.B2[id] -= d3E1 - d1E3;
  f.B3[id] -= d1E2 - d2E1;
}

// E += dt (curl- B - J) and clear J for the next deposit.
// ax.c[l] = C_l dt / dx1; e2 = dt / dx2; e3 = dt / dx3.  J1 is read from
// J1src (the corrected copy for the customized solver).
template <typename Real, int DIM, int MM>
__global__ __launch_bounds__(256) void k_efull(Geo g, Fields<Real> f, const Real *J1src, Axial<Real> ax, Real e2,
                                               Real e3, Real dt) {
  const int l1 = blockIdx.x * blockDim.x + threadIdx.x;
  if (l1 >= g.n1) return;
  const int i2 = blockIdx.y, i3 = blockIdx.z;
  const int s1 = col_of(g, l1);
  const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
  const long long id = row + s1;
  const long long row2m = (long long)g.n1 * (wrap(i2 - 1, g.n2) + (long long)g.n2 * i3);
  const int M = MM > 0 ? MM : ax.M;

  Real d1B3 = 0, d1B2 = 0;
  auto term = [&](int l) {
    const int a = col_of(g, l1 + l - 1), b = col_of(g, l1 - l);
    d1B3 += ax.c[l - 1] * (ld(f.B3, row, a) - ld(f.B3, row, b));
    d1B2 += ax.c[l - 1] * (ld(f.B2, row, a) - ld(f.B2, row, b));
  };
  if (MM > 0) {
#pragma unroll
    for (int l = 1; l <= MM; ++l) term(l);
  } else {
    for (int l = 1; l <= M; ++l) term(l);
  }
  const Real B1 = f.B1[id], B2 = f.B2[id], B3 = f.B3[id];
  const Real d2B3 = e2 * (B3 - f.B3[row2m + s1]);
  const Real d2B1 = e2 * (B1 - f.B1[row2m + s1]);
  Real d3B2 = 0, d3B1 = 0;
  if (DIM == 3) {
    const long long row3m = (long long)g.n1 * (i2 + (long long)g.n2 * wrap(i3 - 1, g.n3));
    d3B2 = e3 * (B2 - f.B2[row3m + s1]);
    d3B1 = e3 * (B1 - f.B1[row3m + s1]);
  }
  const Real j1 = J1src[id], j2 = f.J2[id], j3 = f.J3[id];
  f.E1[id] += d2B3 - d3B2 - dt * j1;
  f.E2[id] += d3B1 - d1B3 - dt * j2;
  f.E3[id] += d1B2 - d2B1 - dt * j3;
  f.J1[id] = Real(0);
  f.J2[id] = Real(0);
  f.J3[id] = Real(0);
}

// J1c = G * J1 along x1: FIR with taps g_0..g_ng (even in m), zero outside
// the window or wrapped on a periodic line.  One block per (segment, row);
// the segment plus its halo is staged in LDS.
constexpr int kCorrSeg = 256;

template <typename Real>
__global__ __launch_bounds__(kCorrSeg) void k_jcorr(Geo g, const Real *J1, Real *J1c, const Real *taps, int ng) {
  __shared__ Real line[kCorrSeg + 2 * kMaxTaps];
  const int l0 = blockIdx.x * kCorrSeg;
  const int i2 = blockIdx.y, i3 = blockIdx.z;
  const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
  const int span = kCorrSeg + 2 * ng;
  for (int t = threadIdx.x; t < span; t += blockDim.x) line[t] = ld(J1, row, col_of(g, l0 - ng + t));
  __syncthreads();
  const int l1 = l0 + threadIdx.x;
  if (l1 >= g.n1) return;
  Real acc = taps[0] * line[threadIdx.x + ng];
  for (int m = 1; m <= ng; ++m) acc += taps[m] * (line[threadIdx.x + ng - m] + line[threadIdx.x + ng + m]);
  J1c[row + col_of(g, l1)] = acc;
}

// Zero the storage column `col` of the given arrays (new leading slab after a
// window shift).
template <typename Real>
__global__ void k_zero_column(Geo g, Fields<Real> f, int col) {
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long rows = (long long)g.n2 * g.n3;
  if (r >= rows) return;
  const long long id = r * g.n1 + col;
  f.E1[id] = f.E2[id] = f.E3[id] = Real(0);
  f.B1[id] = f.B2[id] = f.B3[id] = Real(0);
}

// ---- launchers ---------------------------------------------------------------

template <typename Real, int DIM>
static void bhalf_dispatch(const Geo &g, const Fields<Real> &f, const Axial<Real> &ax, Real h2, Real h3,
                           hipStream_t st) {
  dim3 grid((g.n1 + 255) / 256, g.n2, g.n3);
  if (ax.M == 1)
    k_bhalf<Real, DIM, 1><<<grid, 256, 0, st>>>(g, f, ax, h2, h3);
  else if (ax.M == 16)
    k_bhalf<Real, DIM, 16><<<grid, 256, 0, st>>>(g, f, ax, h2, h3);
  else
    k_bhalf<Real, DIM, 0><<<grid, 256, 0, st>>>(g, f, ax, h2, h3);
}

template <typename Real, int DIM>
static void efull_dispatch(const Geo &g, const Fields<Real> &f, const Real *J1src, const Axial<Real> &ax, Real e2,
                           Real e3, Real dt, hipStream_t st) {
  dim3 grid((g.n1 + 255) / 256, g.n2, g.n3);
  if (ax.M == 1)
    k_efull<Real, DIM, 1><<<grid, 256, 0, st>>>(g, f, J1src, ax, e2, e3, dt);
  else if (ax.M == 16)
    k_efull<Real, DIM, 16><<<grid, 256, 0, st>>>(g, f, J1src, ax, e2, e3, dt);
  else
    k_efull<Real, DIM, 0><<<grid, 256, 0, st>>>(g, f, J1src, ax, e2, e3, dt);
}

template <typename Real>
void launch_bhalf(int ndim, const Geo &g, const Fields<Real> &f, const Axial<Real> &ax, Real h2, Real h3,
                  hipStream_t st) {
  if (ndim == 3)
    bhalf_dispatch<Real, 3>(g, f, ax, h2, h3, st);
  else
    bhalf_dispatch<Real, 2>(g, f, ax, h2, h3, st);
}

template <typename Real>
void launch_efull(int ndim, const Geo &g, const Fields<Real> &f, const Real *J1src, const Axial<Real> &ax, Real e2,
                  Real e3, Real dt, hipStream_t st) {
  if (ndim == 3)
    efull_dispatch<Real, 3>(g, f, J1src, ax, e2, e3, dt, st);
  else
    efull_dispatch<Real, 2>(g, f, J1src, ax, e2, e3, dt, st);
}

template <typename Real>
void launch_jcorr(const Geo &g, const Real *J1, Real *J1c, const Real *taps, int ng, hipStream_t st) {
  dim3 grid((g.n1 + kCorrSeg - 1) / kCorrSeg, g.n2, g.n3);
  k_jcorr<Real><<<grid, kCorrSeg, 0, st>>>(g, J1, J1c, taps, ng);
}

template <typename Real>
void launch_zero_column(const Geo &g, const Fields<Real> &f, int col, hipStream_t st) {
  const long long rows = (long long)g.n2 * g.n3;
  k_zero_column<Real><<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(g, f, col);
}

#define RELPIC_INST_FIELD(Real)                                                                                    \
  template void launch_bhalf<Real>(int, const Geo &, const Fields<Real> &, const Axial<Real> &, Real, Real,        \
                                   hipStream_t);                                                                   \
  template void launch_efull<Real>(int, const Geo &, const Fields<Real> &, const Real *, const Axial<Real> &, Real, \
                                   Real, Real, hipStream_t);                                                       \
  template void launch_jcorr<Real>(const Geo &, const Real *, Real *, const Real *, int, hipStream_t);             \
  template void launch_zero_column<Real>(const Geo &, const Fields<Real> &, int, hipStream_t);

RELPIC_INST_FIELD(float)
RELPIC_INST_FIELD(double)

}  // namespace relpic
