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

// LDS pitch of one staged row of a SEG-cell tile (cells plus the axial halo)
template <int SEG>
constexpr int stage_pitch() {
  return SEG + 2 * kMaxM;
}

// 2D updates that march along x2: one x1 segment [l0, l0 + SEG) of rows
// r0 .. r1 - 1, one thread per x1 cell (blockDim.x == SEG).  The x2
// neighbour the previous row already loaded is carried in registers (E at
// i2 + 1 becomes the next row's own E for the B update; B at i2 becomes the
// next row's i2 - 1 for the E update), and the next row's staged x1 segment
// and the own cell's operands are loaded while the current row is computed.
// Every barrier is reached by all threads.  The LDS arguments hold
// stage_pitch<SEG>() values each.

// Bout = Bin - curl+ E (2D; ax.c[l] = C_l c / dx1, h2 = c / dx2)
template <typename Real, int MM, int SEG>
__device__ __forceinline__ void curl_e_rows(const Geo &g, const Real *E1, const Real *E2, const Real *E3,
                                            const Real *Bin1, const Real *Bin2, const Real *Bin3, Real *Bout1,
                                            Real *Bout2, Real *Bout3, const Axial<Real> &ax, Real h2, int l0, int r0,
                                            int r1, Real *sE2, Real *sE3) {
  const int M = MM > 0 ? MM : ax.M;
  const int l1 = l0 + (int)threadIdx.x;
  const int s1 = l1 < g.n1 ? col_near(g, l1) : -1;
  const bool own = s1 >= 0;
  const int c = (int)threadIdx.x + M - 1;  // LDS index of cell l1
  const int ta = threadIdx.x, tb = threadIdx.x + SEG;
  const bool hb = tb < SEG + 2 * M;
  const int ca = col_of(g, l0 - M + 1 + ta), cb = hb ? col_of(g, l0 - M + 1 + tb) : -1;
  Real pa2, pa3, pb2, pb3;                           // staged E2, E3 of the row
  Real e1u = 0, e3u = 0, q1 = 0, q2 = 0, q3 = 0;     // own cell's operands
  auto fetch = [&](int i2) {
    const long long row = (long long)g.n1 * i2;
    pa2 = ldc(E2, row, ca);
    pa3 = ldc(E3, row, ca);
    pb2 = ldc(E2, row, cb);
    pb3 = ldc(E3, row, cb);
    if (own) {
      const long long id = row + s1, up = (long long)g.n1 * wrap_near(i2 + 1, g.n2) + s1;
      e1u = E1[up];
      e3u = E3[up];
      q1 = Bin1[id];
      q2 = Bin2[id];
      q3 = Bin3[id];
    }
  };
  Real e1 = own ? E1[(long long)g.n1 * r0 + s1] : Real(0);
  fetch(r0);
  for (int i2 = r0; i2 < r1; ++i2) {
    sE2[ta] = pa2;
    sE3[ta] = pa3;
    if (hb) {
      sE2[tb] = pb2;
      sE3[tb] = pb3;
    }
    const Real ce1u = e1u, ce3u = e3u, cq1 = q1, cq2 = q2, cq3 = q3;
    __syncthreads();
    if (i2 + 1 < r1) fetch(i2 + 1);
    if (own) {
      const long long id = (long long)g.n1 * i2 + s1;
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
      const Real e3 = sE3[c];
      const Real d2E3 = h2 * (ce3u - e3);
      const Real d2E1 = h2 * (ce1u - e1);
      Bout1[id] = cq1 - d2E3;
      Bout2[id] = cq2 + d1E3;
      Bout3[id] = cq3 - (d1E2 - d2E1);
      e1 = ce1u;
    }
    __syncthreads();
  }
}

// E += curl- B (2D; ax.c[l] = C_l dt / dx1, e2 = dt / dx2)
template <typename Real, int MM, int SEG>
__device__ __forceinline__ void curl_b_rows(const Geo &g, Real *E1, Real *E2, Real *E3, const Real *B1,
                                            const Real *B2, const Real *B3, const Axial<Real> &ax, Real e2, int l0,
                                            int r0, int r1, Real *sB2, Real *sB3) {
  const int M = MM > 0 ? MM : ax.M;
  const int l1 = l0 + (int)threadIdx.x;
  const int s1 = l1 < g.n1 ? col_near(g, l1) : -1;
  const bool own = s1 >= 0;
  const int c = (int)threadIdx.x + M;  // LDS index of cell l1
  const int ta = threadIdx.x, tb = threadIdx.x + SEG;
  const bool hb = tb < SEG + 2 * M;
  const int ca = col_of(g, l0 - M + ta), cb = hb ? col_of(g, l0 - M + tb) : -1;
  Real pa2, pa3, pb2, pb3;                           // staged B2, B3 of the row
  Real b1 = 0, x1 = 0, x2 = 0, x3 = 0;               // own cell's operands
  auto fetch = [&](int i2) {
    const long long row = (long long)g.n1 * i2;
    pa2 = ldc(B2, row, ca);
    pa3 = ldc(B3, row, ca);
    pb2 = ldc(B2, row, cb);
    pb3 = ldc(B3, row, cb);
    if (own) {
      const long long id = row + s1;
      b1 = B1[id];
      x1 = E1[id];
      x2 = E2[id];
      x3 = E3[id];
    }
  };
  Real b1m = Real(0), b3m = Real(0);
  if (own) {
    const long long dn = (long long)g.n1 * wrap_near(r0 - 1, g.n2) + s1;
    b1m = B1[dn];
    b3m = B3[dn];
  }
  fetch(r0);
  for (int i2 = r0; i2 < r1; ++i2) {
    sB2[ta] = pa2;
    sB3[ta] = pa3;
    if (hb) {
      sB2[tb] = pb2;
      sB3[tb] = pb3;
    }
    const Real cb1 = b1, cx1 = x1, cx2 = x2, cx3 = x3;
    __syncthreads();
    if (i2 + 1 < r1) fetch(i2 + 1);
    if (own) {
      const long long id = (long long)g.n1 * i2 + s1;
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
      const Real b3 = sB3[c];
      const Real d2B3 = e2 * (b3 - b3m);
      const Real d2B1 = e2 * (cb1 - b1m);
      E1[id] = cx1 + d2B3;
      E2[id] = cx2 - d1B3;
      E3[id] = cx3 + (d1B2 - d2B1);
      b1m = cb1;
      b3m = b3;
    }
    __syncthreads();
  }
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

// J cleared over the deposit box (x1 widened by pad)
template <typename Real>
__device__ __forceinline__ void clear_j_box(const Geo &g, Real *J1, Real *J2, Real *J3, const JBox &b, int pad,
                                            long long t0, long long stride) {
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
