// Internal types shared by the HIP kernels and the host engine of relpic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace relpic {

constexpr int kMaxM = 32;      // longest axial stencil (2M points)
constexpr int kMaxTaps = 64;   // half-width bound of the J1 correction FIR

// Division of n < 2^31 by a fixed divisor d >= 1 as a multiply-high, add
// and shift (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): with L = ceil(log2 d) and
// m = floor(2^32 (2^L - d) / d) + 1 < 2^32, n / d = (mulhi(m, n) + n) >> L.
struct FastDiv {
  unsigned m;
  int L;
};

__host__ __device__ inline FastDiv make_fastdiv(unsigned d) {
  int L = 0;
  while ((1ull << L) < d) ++L;
  FastDiv f;
  f.m = (unsigned)((((1ull << 32) * ((1ull << L) - d)) / d) + 1);
  f.L = L;
  return f;
}

__device__ __forceinline__ unsigned fdiv(const FastDiv &f, unsigned n) { return (__umulhi(f.m, n) + n) >> f.L; }

// Grid geometry as the kernels see it.  x1 storage is a ring buffer: the
// storage column of global cell g is g mod n1, window cell l lives at
// (l + ws_mod) mod n1.
struct Geo {
  int n1, n2, n3;  // n3 = 1 in 2D
  int ws_mod;      // window start mod n1 (0 when periodic)
  int window;      // 1: values outside window cells [0, n1) read as zero
  int pad_;
  long long N;     // n1 * n2 * n3
  FastDiv dv1, dv2;  // division by n1 and by n2
};

// packed storage index -> (storage column, x2 cell, x3 cell)
__device__ __forceinline__ void unpack_cell(const Geo &g, int packed, int &s1, int &c2, int &c3) {
  const unsigned q1 = fdiv(g.dv1, (unsigned)packed);
  const unsigned q2 = fdiv(g.dv2, q1);
  s1 = packed - (int)q1 * g.n1;
  c2 = (int)q1 - (int)q2 * g.n2;
  c3 = (int)q2;
}

template <typename Real>
struct Fields {
  Real *E1, *E2, *E3, *B1, *B2, *B3, *J1, *J2, *J3;
  Real *J1c;  // corrected J1 (customized solver), scratch
};

// Axial stencil with the 1/dx1 and time-step factors folded in.
template <typename Real>
struct Axial {
  int M;
  Real c[kMaxM];
};

// The second B buffer (B at the other half-integer time).
template <typename Real>
struct HalfB {
  const Real *B1, *B2, *B3;
};

template <typename Real>
struct Particles {
  int *cell;  // packed storage index s1 + n1 * (s2 + n2 * s3); -1 = dropped
  Real *o1, *o2, *o3;
  Real *u1, *u2, *u3;
  long long n;
};

// window-cell index -> storage column, or -1 outside the window
__device__ __forceinline__ int col_of(const Geo &g, int l) {
  if (g.window) {
    if (l < 0 || l >= g.n1) return -1;
    int s = l + g.ws_mod;
    return s >= g.n1 ? s - g.n1 : s;
  }
  int s = l + g.ws_mod;
  if (s >= -g.n1 && s < 2 * g.n1) return s < 0 ? s + g.n1 : (s >= g.n1 ? s - g.n1 : s);
  s %= g.n1;  // far outside: general wrap
  return s < 0 ? s + g.n1 : s;
}

__device__ __forceinline__ int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// wrap for indices known to lie in [-n, 2n)
__device__ __forceinline__ int wrap_near(int i, int n) {
  i = i < 0 ? i + n : i;
  return i >= n ? i - n : i;
}

// col_of for window cells within one grid length of the window ([-n1, 2 n1))
__device__ __forceinline__ int col_near(const Geo &g, int l) {
  if (g.window && (l < 0 || l >= g.n1)) return -1;
  return wrap_near(l + g.ws_mod, g.n1);
}

// Current bounding box of deposited J: window x1 and wrapped x2, x3 (min, max).
struct JBox {
  int lo[3], hi[3];
};

}  // namespace relpic
