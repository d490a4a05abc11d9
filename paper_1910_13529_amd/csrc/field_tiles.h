// Field-advance device code shared by the single-run and batched kernels
// (internal to relpic).
#pragma once

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

// LDS pitch of one staged row of a SEG-cell tile (cells plus the axial halo)
template <int SEG>
constexpr int stage_pitch() {
  return SEG + 2 * kMaxM;
}

// Bout = Bin - curl+ E on a tile of ROWS x1-segments [l0, l0 + SEG) of rows
// i2 .. i2 + ROWS - 1 (those below n2) in plane i3; blockDim.x == SEG * ROWS,
// thread t takes cell l0 + t % SEG of row i2 + t / SEG.  Coefficients carry
// the time factor: ax.c[l] = C_l c / dx1, h2 = c / dx2, h3 = c / dx3.  sE2,
// sE3: LDS of ROWS * stage_pitch<SEG>() values.  Contains one barrier that
// every thread of the workgroup reaches.
template <typename Real, int DIM, int MM, int SEG, int ROWS>
__device__ __forceinline__ void curl_e_tile(const Geo &g, const Real *E1, const Real *E2, const Real *E3,
                                            const Real *Bin1, const Real *Bin2, const Real *Bin3, Real *Bout1,
                                            Real *Bout2, Real *Bout3, const Axial<Real> &ax, Real h2, Real h3, int l0,
                                            int i2, int i3, Real *sE2, Real *sE3) {
  const int M = MM > 0 ? MM : ax.M;
  const int tx = ROWS == 1 ? (int)threadIdx.x : (int)threadIdx.x % SEG;
  const int ty = ROWS == 1 ? 0 : (int)threadIdx.x / SEG;
  i2 += ty;
  const bool live_row = ROWS == 1 || i2 < g.n2;
  sE2 += ty * stage_pitch<SEG>();
  sE3 += ty * stage_pitch<SEG>();
  const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
  // stage E2, E3 on window cells [l0 - M + 1, l0 + SEG + M)
  const int span = SEG + 2 * M;
  if (live_row)
    for (int t = tx; t < span; t += SEG) {
      const int col = col_of(g, l0 - M + 1 + t);
      sE2[t] = ldc(E2, row, col);
      sE3[t] = ldc(E3, row, col);
    }
  __syncthreads();
  const int l1 = l0 + tx;
  if (!live_row || l1 >= g.n1) return;
  const int s1 = col_near(g, l1);
  const long long id = row + s1;
  const int c = tx + M - 1;  // LDS index of cell l1
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
  const Real e1 = E1[id], e2 = sE2[c], e3 = sE3[c];
  const Real d2E3 = h2 * (E3[row2p + s1] - e3);
  const Real d2E1 = h2 * (E1[row2p + s1] - e1);
  Real d3E2 = 0, d3E1 = 0;
  if (DIM == 3) {
    const long long row3p = (long long)g.n1 * (i2 + (long long)g.n2 * wrap_near(i3 + 1, g.n3));
    d3E2 = h3 * (E2[row3p + s1] - e2);
    d3E1 = h3 * (E1[row3p + s1] - e1);
  }
  Bout1[id] = Bin1[id] - (d2E3 - d3E2);
  Bout2[id] = Bin2[id] - (d3E1 - d1E3);
  Bout3[id] = Bin3[id] - (d1E2 - d2E1);
}

// E += curl- B on a tile laid out as in curl_e_tile (ax.c[l] = C_l dt / dx1;
// e2 = dt / dx2; e3 = dt / dx3).  sB2, sB3: LDS of ROWS * stage_pitch<SEG>().
template <typename Real, int DIM, int MM, int SEG, int ROWS>
__device__ __forceinline__ void curl_b_tile(const Geo &g, Real *E1, Real *E2, Real *E3, const Real *B1,
                                            const Real *B2, const Real *B3, const Axial<Real> &ax, Real e2, Real e3,
                                            int l0, int i2, int i3, Real *sB2, Real *sB3) {
  const int M = MM > 0 ? MM : ax.M;
  const int tx = ROWS == 1 ? (int)threadIdx.x : (int)threadIdx.x % SEG;
  const int ty = ROWS == 1 ? 0 : (int)threadIdx.x / SEG;
  i2 += ty;
  const bool live_row = ROWS == 1 || i2 < g.n2;
  sB2 += ty * stage_pitch<SEG>();
  sB3 += ty * stage_pitch<SEG>();
  const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
  // stage B2, B3 on window cells [l0 - M, l0 + SEG + M)
  const int span = SEG + 2 * M;
  if (live_row)
    for (int t = tx; t < span; t += SEG) {
      const int col = col_of(g, l0 - M + t);
      sB2[t] = ldc(B2, row, col);
      sB3[t] = ldc(B3, row, col);
    }
  __syncthreads();
  const int l1 = l0 + tx;
  if (!live_row || l1 >= g.n1) return;
  const int s1 = col_near(g, l1);
  const long long id = row + s1;
  const int c = tx + M;  // LDS index of cell l1
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
  const Real b1 = B1[id], b2 = sB2[c], b3 = sB3[c];
  const Real d2B3 = e2 * (b3 - B3[row2m + s1]);
  const Real d2B1 = e2 * (b1 - B1[row2m + s1]);
  Real d3B2 = 0, d3B1 = 0;
  if (DIM == 3) {
    const long long row3m = (long long)g.n1 * (i2 + (long long)g.n2 * wrap_near(i3 - 1, g.n3));
    d3B2 = e3 * (b2 - B2[row3m + s1]);
    d3B1 = e3 * (b1 - B1[row3m + s1]);
  }
  E1[id] += d2B3 - d3B2;
  E2[id] += d3B1 - d1B3;
  E3[id] += d1B2 - d2B1;
}

// Window-cell range of the deposit box along x1 widened by pad (clamped to
// the window, or the whole periodic line).  Returns false for an empty box.
__device__ __forceinline__ bool box_x1(const Geo &g, const JBox &b, int pad, int &lo1, int &hi1) {
  if (b.hi[0] < b.lo[0]) return false;
  lo1 = b.lo[0] - pad;
  hi1 = b.hi[0] + pad;
  if (g.window) {
    lo1 = lo1 < 0 ? 0 : lo1;
    hi1 = hi1 > g.n1 - 1 ? g.n1 - 1 : hi1;
  } else if (hi1 - lo1 + 1 >= g.n1) {
    lo1 = 0;
    hi1 = g.n1 - 1;
  }
  return true;
}

// E -= dt J over the deposit box (x1 widened by pad), J cleared there; work
// items t0, t0 + stride, ...
template <typename Real>
__device__ __forceinline__ void add_j_box(const Geo &g, Real *E1, Real *E2, Real *E3, Real *J1, Real *J2, Real *J3,
                                          const Real *J1src, Real dt, const JBox &b, int pad, long long t0,
                                          long long stride) {
  int lo1, hi1;
  if (!box_x1(g, b, pad, lo1, hi1)) return;
  const long long w1 = hi1 - lo1 + 1, w2 = b.hi[1] - b.lo[1] + 1, w3 = b.hi[2] - b.lo[2] + 1;
  const long long tot = w1 * w2 * w3;
  for (long long t = t0; t < tot; t += stride) {
    const int a = (int)(t % w1);
    const long long r = t / w1;
    const int i2 = b.lo[1] + (int)(r % w2);
    const int i3 = b.lo[2] + (int)(r / w2);
    const long long id = (long long)g.n1 * (i2 + (long long)g.n2 * i3) + col_of(g, lo1 + a);
    E1[id] -= dt * J1src[id];
    E2[id] -= dt * J2[id];
    E3[id] -= dt * J3[id];
    J1[id] = Real(0);
    J2[id] = Real(0);
    J3[id] = Real(0);
  }
}

// J1c = G * J1 along x1 inside the deposit box (x1 widened by ng)
template <typename Real>
__device__ __forceinline__ void jcorr_box(const Geo &g, const Real *J1, Real *J1c, const Real *taps, int ng,
                                          const JBox &b, long long t0, long long stride) {
  int lo1, hi1;
  if (!box_x1(g, b, ng, lo1, hi1)) return;
  const long long w1 = hi1 - lo1 + 1, w2 = b.hi[1] - b.lo[1] + 1, w3 = b.hi[2] - b.lo[2] + 1;
  const long long tot = w1 * w2 * w3;
  for (long long t = t0; t < tot; t += stride) {
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

}  // namespace relpic
