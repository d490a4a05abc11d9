// Particle phase device code shared by the single-run and batched kernels
// (internal to relpic).
#pragma once

#include <climits>

#include "kernels.h"
#include "xlane.h"

namespace relpic {

constexpr int kPushBlock = 256;
constexpr int kTileBytes = 49152;  // LDS tile per workgroup: J (3 components) + E, B (6)
// The single-run FP32 push runs three workgroups per CU in 160 KB of LDS
// (tile, box words and cell-group tables of each within a third); the FP64
// push two waves per SIMD (two workgroups per CU), which leaves room for 768
// cells of 9 FP64 words.
template <typename Real>
struct PushTile {
  static constexpr int bytes = 52224;
};
template <>
struct PushTile<double> {
  static constexpr int bytes = 61440;
};
constexpr int kChunkBoxInts = 10;  // LDS words of a chunk's box: min/max per axis, tile dividers

typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) double lds_f64;

// atomic add to a workgroup-shared (LDS) address: ds_add_f32 / ds_add_f64
__device__ __forceinline__ void lds_add(float *p, float v) {
  __hip_atomic_fetch_add((lds_f32 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(double *p, double v) {
  __hip_atomic_fetch_add((lds_f64 *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// load from a workgroup-shared (LDS) address
__device__ __forceinline__ float lds_ld(const float *p) { return *(const lds_f32 *)p; }
__device__ __forceinline__ double lds_ld(const double *p) { return *(const lds_f64 *)p; }


// 1/sqrt(x) and 1/x for the Boris push: the hardware reciprocal square root
// and reciprocal in FP32 (about one ulp, against the several instructions of
// a correctly rounded division or square root), exact operations in FP64.
template <typename Real>
__device__ __forceinline__ Real push_rsqrt(Real x) {
  return Real(1) / sqrt(x);
}
template <>
__device__ __forceinline__ float push_rsqrt<float>(float x) {
  return __builtin_amdgcn_rsqf(x);
}
template <typename Real>
__device__ __forceinline__ Real push_rcp(Real x) {
  return Real(1) / x;
}
template <>
__device__ __forceinline__ float push_rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// quadratic B-spline weights at nodes -1, 0, +1 for a particle at offset d
// from node 0 (d in [-1/2, 1/2])
template <typename Real>
__device__ __forceinline__ void qw(Real d, Real w[3]) {
  const Real a = Real(0.5) - d, b = Real(0.5) + d;
  w[0] = Real(0.5) * a * a;
  w[1] = Real(0.75) - d * d;
  w[2] = Real(0.5) * b * b;
}

// Weights for a component at half-integer points j + 1/2: returns the index
// j of the middle point and its weights.
template <typename Real>
__device__ __forceinline__ int qw_half(int c, Real o, Real w[3]) {
  // the offset from the nearer half point is selected first, so one set of
  // weights is evaluated (not both branches and a select of each weight)
  const bool up = o >= Real(0);
  qw(up ? o - Real(0.5) : o + Real(0.5), w);
  return up ? c : c - 1;
}

// Gather stencils of one particle: element offsets of the x1 columns and of
// the x2 (n1 * i2) and x3 (n1 * n2 * i3) rows, for node (N) and half-integer
// (H) points, and the weights.  Offsets are 32-bit (the library keeps every
// field array below 4 GiB) so loads take a scalar base plus one vector
// offset; x1 points outside the moving window carry weight 0 and a valid
// dummy column.
template <typename Real>
struct Stagger {
  unsigned colN[3], colH[3];
  unsigned rowN2[3], rowH2[3], rowN3[3], rowH3[3];
  Real wN[3][3], wH[3][3];
};

// Element j of a particle array through a 32-bit byte offset from its base
// (a species holds at most 2^32 bytes per array), so loads and stores take
// a scalar base and one vector offset.
template <typename T>
__device__ __forceinline__ T &el32(T *base, unsigned j) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + j * (unsigned)sizeof(T));
}

// Load element `id` through a 32-bit byte offset from the array base.
template <typename Real>
__device__ __forceinline__ Real ld32(const Real *__restrict__ f, unsigned id) {
  return *reinterpret_cast<const Real *>(reinterpret_cast<const char *>(f) + (unsigned)(id * (unsigned)sizeof(Real)));
}

template <typename Real, int DIM, bool H1, bool H2, bool H3, bool AVG>
__device__ __forceinline__ Real interp(const Stagger<Real> &s, const Real *__restrict__ f,
                                       const Real *__restrict__ f2) {
  const unsigned *cols = H1 ? s.colH : s.colN;
  const unsigned *r2 = H2 ? s.rowH2 : s.rowN2;
  Real acc = 0;
  if (DIM == 2) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Real r = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const unsigned id = r2[b] + cols[a];
        const Real v = AVG ? ld32(f, id) + ld32(f2, id) : ld32(f, id);
        r += (H1 ? s.wH[0][a] : s.wN[0][a]) * v;
      }
      acc += (H2 ? s.wH[1][b] : s.wN[1][b]) * r;
    }
  } else {
    const unsigned *r3 = H3 ? s.rowH3 : s.rowN3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Real rc = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Real r = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const unsigned id = r2[b] + r3[c] + cols[a];
          const Real v = AVG ? ld32(f, id) + ld32(f2, id) : ld32(f, id);
          r += (H1 ? s.wH[0][a] : s.wN[0][a]) * v;
        }
        rc += (H2 ? s.wH[1][b] : s.wN[1][b]) * r;
      }
      acc += (H3 ? s.wH[2][c] : s.wN[2][c]) * rc;
    }
  }
  return AVG ? Real(0.5) * acc : acc;
}

// Gather from the workgroup's LDS copy of E and B (B already averaged to
// integer time): tile offsets of the x1 cells c-2 .. c+1 and of the x2/x3
// rows c-2 .. c+1 (scaled by the tile strides).
struct StaggerL {
  int x1[4], x2[4], x3[4];
  bool h1lo, h2lo, h3lo;
};

// The stencil of each staggering starts at one of two consecutive window
// cells per axis (x1[k + 1] = x1[k] + 1, likewise x2, x3 in rows and
// planes), so one start per axis is selected and the three cells of an x1
// row are read at constant offsets from one address.
template <typename Real, int DIM, bool H1, bool H2, bool H3>
__device__ __forceinline__ Real interp_lds(const StaggerL &s, const Real wN[3][3], const Real wH[3][3],
                                           const Real *ft) {
  const int x0 = (H1 && s.h1lo) ? s.x1[0] : s.x1[1];
  const int y0 = (H2 && s.h2lo) ? s.x2[0] : s.x2[1];
  const int dy = s.x2[1] - s.x2[0];
  const int z0 = DIM == 3 ? ((H3 && s.h3lo) ? s.x3[0] : s.x3[1]) : 0;
  const int dz = DIM == 3 ? s.x3[1] - s.x3[0] : 0;
  // one lane pointer per component; the row and plane steps are the same
  // for every component, so they stay a few uniform offsets
  const Real *p0 = ft + (x0 + y0 + z0);
  Real acc = 0;
#pragma unroll
  for (int c = 0; c < (DIM == 3 ? 3 : 1); ++c) {
    Real rc = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const Real *row = p0 + (b * dy + c * dz);
      Real r = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) r += (H1 ? wH[0][a] : wN[0][a]) * lds_ld(row + a);
      rc += (H2 ? wH[1][b] : wN[1][b]) * r;
    }
    acc += DIM == 3 ? (H3 ? wH[2][c] : wN[2][c]) * rc : rc;
  }
  return acc;
}

// Esirkepov shape arrays on four nodes starting at old cell + base:
// S0 at x^n, DS = S(x^{n+1}) - S(x^n); cum = running sum of DS.
// The cell moves by sh in {-1, 0, 1}.  Node base + a (a = 0..3) relative to
// the old cell, base = -2 when the particle moved down a cell, else -1: the
// old weights sit on a = 0..2, or on a = 1..3 after a move down; the new
// ones (node base + a - sh of the new cell) on a = 0..2, or on a = 1..3
// after a move up.  Selecting with the two flags (rather than comparing
// every node index) keeps the number of lane masks, and of the scalar
// registers holding them, at two.
template <typename Real>
__device__ __forceinline__ int esirkepov_1d(Real o0, int sh, Real o1, Real S0[4], Real DS[4], Real cum[4]) {
  Real w0[3], w1[3];
  qw(o0, w0);
  qw(o1, w1);
  const bool dn = sh < 0, up = sh > 0;
  const Real s0[4] = {dn ? Real(0) : w0[0], dn ? w0[0] : w0[1], dn ? w0[1] : w0[2], dn ? w0[2] : Real(0)};
  const Real s1[4] = {up ? Real(0) : w1[0], up ? w1[0] : w1[1], up ? w1[1] : w1[2], up ? w1[2] : Real(0)};
  Real run = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    S0[a] = s0[a];
    DS[a] = s1[a] - s0[a];
    run += DS[a];
    cum[a] = run;
  }
  return dn ? -2 : -1;
}

// Where deposits go: the workgroup's LDS tile if it covers the point, else
// J in HBM.  Coordinates are the window x1 index and unwrapped x2, x3.  An
// FP32 run accumulates the tile's current in FP64 (tile_d) when the tile has
// room: LDS atomic adds of FP64 words take a few cycles per wavefront
// instruction on gfx950, those of FP32 words about three cycles per lane.
template <typename Real>
struct Sink {
  Real *tile;        // 3 components x T1 x T2 x T3, or null
  double *tile_d;    // the current as FP64 words (an FP32 run that fits them; an FP64 run: tile), or null
  int t1, t2, t3;    // tile origin
  int T1, T2, T3;    // tile extents
  int tn;            // T1 * T2 * T3
  Real *J[3];
  Geo g;

  __device__ __forceinline__ void add(int comp, int x1, int x2, int x3, Real v) const {
    if (v == Real(0)) return;
    if (tile) {
      const int a = x1 - t1, b = x2 - t2, c = x3 - t3;
      if (a >= 0 && a < T1 && b >= 0 && b < T2 && c >= 0 && c < T3) {
        const int id = comp * tn + a + T1 * (b + T2 * c);
        if (tile_d)
          lds_add(tile_d + id, (double)v);
        else
          lds_add(tile + id, v);
        return;
      }
    }
    const int col = col_near(g, x1);
    if (col < 0) return;
    const long long row = (long long)g.n1 * (wrap_near(x2, g.n2) + (long long)g.n2 * wrap_near(x3, g.n3));
    atomicAdd(J[comp] + row + col, v);
  }
};

// One level of the reduce-scatter: v[0..S) is summed with the partner lane
// (lane ^ BIT); lanes with the bit set keep the upper half.
template <typename Real, int S, int BIT>
__device__ __forceinline__ void rs_level(Real *v, int lane, int &off) {
  constexpr int H = (S + 1) / 2;
  const bool up = (lane & BIT) != 0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    Real lo = v[j];
    Real hi = (j + H < S) ? v[j + H] : Real(0);
    if constexpr (BIT >= 16) {
      // after the swap a lane holds its own kept half and the partner's copy
      // of that half, in either order
      swap_lanes<BIT>(lo, hi);
      v[j] = lo + hi;
    } else {
      const Real send = up ? lo : hi;
      const Real keep = up ? hi : lo;
      v[j] = keep + xor_lane<BIT>(send);
    }
  }
  if (up) off += H;
}

// Sum v[0..S) over the 64 lanes of the wavefront (S <= 64); afterwards each
// lane holds in v[0] the total for index `off` (padding when off >= S).
template <typename Real, int S, int BIT>
__device__ __forceinline__ void reduce_scatter(Real *v, int lane, int &off) {
  if constexpr (BIT >= 1) {
    rs_level<Real, S, BIT>(v, lane, off);
    reduce_scatter<Real, (S + 1) / 2, BIT / 2>(v, lane, off);
  }
}

// minimum / maximum over the wavefront, in every lane
__device__ __forceinline__ int wave_min(int v) {
  v = min(v, xor_lane<32>(v));
  v = min(v, xor_lane<16>(v));
  v = min(v, xor_lane<8>(v));
  v = min(v, xor_lane<4>(v));
  v = min(v, xor_lane<2>(v));
  return min(v, xor_lane<1>(v));
}

__device__ __forceinline__ int wave_max(int v) {
  v = max(v, xor_lane<32>(v));
  v = max(v, xor_lane<16>(v));
  v = max(v, xor_lane<8>(v));
  v = max(v, xor_lane<4>(v));
  v = max(v, xor_lane<2>(v));
  return max(v, xor_lane<1>(v));
}

// Sum an N1 x N2 x N3 box of per-lane values v over the wavefront and add the
// totals (one per lane) to the sink at box origin (x1, x2, x3); v is
// overwritten.
template <typename Real, int N1, int N2, int N3>
__device__ __forceinline__ void box_reduce_add(const Sink<Real> &sk, int comp, int lane, int x1, int x2, int x3,
                                               Real *v) {
  constexpr int S = N1 * N2 * N3;
  static_assert(S <= 64, "box larger than a wavefront");
  int off = 0;
  reduce_scatter<Real, S, 32>(v, lane, off);
  if (off < S) sk.add(comp, x1 + off % N1, x2 + (off / N1) % N2, x3 + off / (N1 * N2), v[0]);
}

// Everything the deposit needs from one pushed particle.
template <typename Real>
struct Moved {
  int c[3];          // old cell (window x1, x2, x3)
  int base[3];       // first stencil node relative to the old cell (-2 or -1)
  Real S0[3][4], DS[3][4], cum[3][4];
  Real jz;           // Q v3 / dV (2D out-of-plane current)
};

template <typename Real>
__device__ __forceinline__ Real wperp(const Real *S0a, const Real *DSa, const Real *S0b, const Real *DSb, int a,
                                      int b) {
  return S0a[a] * S0b[b] + Real(0.5) * DSa[a] * S0b[b] + Real(0.5) * S0a[a] * DSb[b] +
         DSa[a] * DSb[b] * Real(1.0 / 3.0);
}

// Direct Esirkepov deposit of one particle into the sink.
template <typename Real, int DIM>
__device__ __forceinline__ void deposit_direct(const Moved<Real> &m, const PushParams<Real> &q, const Sink<Real> &sk) {
  const int x1 = m.c[0] + m.base[0], x2 = m.c[1] + m.base[1];
  if (DIM == 2) {
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const Real wt = q.f1 * (m.S0[1][bb] + Real(0.5) * m.DS[1][bb]);
#pragma unroll
      for (int aa = 0; aa < 3; ++aa) sk.add(0, x1 + aa, x2 + bb, 0, wt * m.cum[0][aa]);
    }
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) {
      const Real wt = q.f2 * (m.S0[0][aa] + Real(0.5) * m.DS[0][aa]);
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) sk.add(1, x1 + aa, x2 + bb, 0, wt * m.cum[1][bb]);
    }
#pragma unroll
    for (int aa = 0; aa < 4; ++aa)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
        sk.add(2, x1 + aa, x2 + bb, 0, m.jz * wperp(m.S0[0], m.DS[0], m.S0[1], m.DS[1], aa, bb));
  } else {
    const int x3 = m.c[2] + m.base[2];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const Real wt = q.f1 * wperp(m.S0[1], m.DS[1], m.S0[2], m.DS[2], bb, cc);
        if (wt == Real(0)) continue;
#pragma unroll
        for (int aa = 0; aa < 3; ++aa) sk.add(0, x1 + aa, x2 + bb, x3 + cc, wt * m.cum[0][aa]);
      }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        const Real wt = q.f2 * wperp(m.S0[0], m.DS[0], m.S0[2], m.DS[2], aa, cc);
        if (wt == Real(0)) continue;
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) sk.add(1, x1 + aa, x2 + bb, x3 + cc, wt * m.cum[1][bb]);
      }
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        const Real wt = q.f3 * wperp(m.S0[0], m.DS[0], m.S0[1], m.DS[1], aa, bb);
        if (wt == Real(0)) continue;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) sk.add(2, x1 + aa, x2 + bb, x3 + cc, wt * m.cum[2][cc]);
      }
  }
}

// Shift an N-point stencil array into a box frame W - 1 points wider:
// out[b] = in[b - o] (zero outside), o in [0, W).
template <typename Real, int N, int W>
__device__ __forceinline__ Real ext_shift(const Real *in, int o, int b) {
  Real r = Real(0);
#pragma unroll
  for (int sft = 0; sft < W; ++sft) {
    const int j = b - sft;
    if (j >= 0 && j < N) r = (o == sft) ? in[j] : r;
  }
  return r;
}

// Wavefront-collective deposit (every lane of the wave must call it), in
// rounds.  In a round the pending lanes in the (x2, x3) row of the first
// pending lane join the reduction if their x1 stencil starts at most W - 1
// nodes after the leftmost one among them (that lane always joins, so every
// round retires at least one lane).  Their exact supports are then J1: 4 x 3 x 3
// half/node points, J2: 5 x 2 x 3, J3: 5 x 3 x 2 (2D: 4 x 3, 5 x 2, 5 x 3),
// all inside boxes that every such lane shares (3D with W = 4: stencils
// starting up to three nodes after the leftmost one join, in boxes three
// points wider, J1: 6 x 3 x 3, J2: 7 x 2 x 3, J3: 7 x 3 x 2; fewer rounds when
// a wavefront's particles spread over several cells, as in a plasma).  Lanes that cross a
// transverse cell boundary this step (a four-node transverse support) are not
// pending and go to the direct path, which the whole wavefront executes as
// soon as one lane needs it.  In 3D a round costs a fraction of it (144
// stencil points against 96 reduced values), so rounds run until no pending
// lane is left; in 2D (40 points against 37 values) after kDepositRounds2D
// rounds the rest goes direct.  Returns whether this lane's particle still
// has to be deposited directly.
constexpr int kDepositRounds = 64;
constexpr int kDepositRounds2D = 3;

template <typename Real, int DIM, int W = 2>
__device__ __forceinline__ bool deposit_wave(bool active, const Moved<Real> &m, const PushParams<Real> &q,
                                             const Sink<Real> &sk) {
  static_assert(W == 2 || (W == 4 && DIM == 3), "round width");
  constexpr int NX = W + 3;  // x1 nodes of the J2, J3 boxes (J1: NX - 1 half points)
  const int lane = threadIdx.x & 63;
  // no transverse crossing: base -1 and no DS on the fourth node
  const bool flat2 = m.base[1] == -1 && m.DS[1][3] == Real(0);
  const bool flat3 = DIM == 2 || (m.base[2] == -1 && m.DS[2][3] == Real(0));
  bool pending = active && flat2 && flat3;  // candidates for a reduction round
  for (int round = 0; round < (DIM == 3 ? kDepositRounds : kDepositRounds2D); ++round) {
    const unsigned long long act = __ballot(pending);
    if (act == 0ULL) break;
    const int first = __ffsll((long long)act) - 1;
    const int c2w = __builtin_amdgcn_readlane(m.c[1], first);
    const int c3w = __builtin_amdgcn_readlane(m.c[2], first);
    const bool inrow = pending && m.c[1] == c2w && (DIM == 2 || m.c[2] == c3w);
    // leftmost x1 stencil start among them; the lane that has it always fits
    const int smin = wave_min(inrow ? m.c[0] + m.base[0] : INT_MAX);
    const int o1 = m.c[0] + m.base[0] - smin;
    const bool fits = inrow && o1 >= 0 && o1 < W;
    {
      // Branch-free separable form of the exact supports: each box value is an
      // x1 factor (or x2/x3 running sum) times a transverse Esirkepov weight
      //   S0a S0b + DSa S0b/2 + S0a DSb/2 + DSa DSb/3 = S0a P_b + DSa Q_b,
      // P = S0 + DS/2, Q = S0/2 + DS/3; lanes that do not fit contribute 0.
      const int oo = fits ? o1 : 0;
      const Real z = fits ? Real(1) : Real(0);
      Real e1S0[NX], e1DS[NX];
#pragma unroll
      for (int b = 0; b < NX; ++b) {
        e1S0[b] = ext_shift<Real, 4, W>(m.S0[0], oo, b);
        e1DS[b] = ext_shift<Real, 4, W>(m.DS[0], oo, b);
      }
      // J1 at x1 half points: running sum of DS1 (three entries) shifted by oo
      Real c1[NX - 1];
#pragma unroll
      for (int b = 0; b < NX - 1; ++b) c1[b] = z * q.f1 * ext_shift<Real, 3, W>(m.cum[0], oo, b);
      Real P2[3], Q2[3], P3[3], Q3[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        P2[k] = m.S0[1][k] + Real(0.5) * m.DS[1][k];
        Q2[k] = Real(0.5) * m.S0[1][k] + Real(1.0 / 3.0) * m.DS[1][k];
        P3[k] = m.S0[2][k] + Real(0.5) * m.DS[2][k];
        Q3[k] = Real(0.5) * m.S0[2][k] + Real(1.0 / 3.0) * m.DS[2][k];
      }
      const int x1 = smin, x2 = c2w - 1, x3 = DIM == 3 ? c3w - 1 : 0;
      if (DIM == 3) {
        {
          Real v[(NX - 1) * 9];
#pragma unroll
          for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
            for (int a2 = 0; a2 < 3; ++a2) {
              const Real w = m.S0[1][a2] * P3[a3] + m.DS[1][a2] * Q3[a3];
#pragma unroll
              for (int b = 0; b < NX - 1; ++b) v[b + (NX - 1) * (a2 + 3 * a3)] = c1[b] * w;
            }
          box_reduce_add<Real, NX - 1, 3, 3>(sk, 0, lane, x1, x2, x3, v);
        }
        {
          Real v[NX * 6];
#pragma unroll
          for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
            for (int b = 0; b < NX; ++b) {
              const Real w = e1S0[b] * P3[a3] + e1DS[b] * Q3[a3];
#pragma unroll
              for (int a2 = 0; a2 < 2; ++a2) v[b + NX * (a2 + 2 * a3)] = z * q.f2 * m.cum[1][a2] * w;
            }
          box_reduce_add<Real, NX, 2, 3>(sk, 1, lane, x1, x2, x3, v);
        }
        {
          Real v[NX * 6];
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
            for (int b = 0; b < NX; ++b) {
              const Real w = e1S0[b] * P2[a2] + e1DS[b] * Q2[a2];
#pragma unroll
              for (int a3 = 0; a3 < 2; ++a3) v[b + NX * (a2 + 3 * a3)] = z * q.f3 * m.cum[2][a3] * w;
            }
          box_reduce_add<Real, NX, 3, 2>(sk, 2, lane, x1, x2, x3, v);
        }
      } else {
        {
          Real v[12];
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
            for (int b = 0; b < 4; ++b) v[b + 4 * a2] = c1[b] * P2[a2];
          box_reduce_add<Real, 4, 3, 1>(sk, 0, lane, x1, x2, 0, v);
        }
        {
          Real v[10];
#pragma unroll
          for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
            for (int b = 0; b < 5; ++b) v[b + 5 * a2] = z * q.f2 * m.cum[1][a2] * (e1S0[b] + Real(0.5) * e1DS[b]);
          box_reduce_add<Real, 5, 2, 1>(sk, 1, lane, x1, x2, 0, v);
        }
        {
          Real v[15];
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
            for (int b = 0; b < 5; ++b) v[b + 5 * a2] = z * m.jz * (e1S0[b] * P2[a2] + e1DS[b] * Q2[a2]);
          box_reduce_add<Real, 5, 3, 1>(sk, 2, lane, x1, x2, 0, v);
        }
      }
      pending = pending && !fits;
    }
  }
  // lanes left: crossing a transverse boundary, or beyond the rounds
  return active && (pending || !(flat2 && flat3));
}

// ---- cell groups (tile-sorted 3D species) ------------------------------------------
//
// A sorted plasma holds its particles in runs of one cell each (eight per cell
// at 8 ppc), but a run can start anywhere in the array, so aligned lanes do
// not share cells.  A grouped chunk maps each run, cut into pieces of at most
// eight, onto one 8-lane group of a wavefront: group gi of the chunk takes
// lanes 8 (gi mod 32) .. + 7 of iteration gi / 32.  All particles of a group
// then share one cell, and those whose exact supports lie in that cell's
// frame (node base -1 on every axis, no transverse crossing) are summed over
// the group by a three-level reduce-scatter (gfx950 DPP: row half-mirror,
// then lane ^ 1 and lane ^ 2), after which each of the eight lanes adds ten
// of the frame's 75 points to the LDS tile.

constexpr int kGroupMax = 32 * 9;  // groups of a grouped chunk (<= 2048 particles, <= 9 iterations)
constexpr int kGroupSlots = 80;    // 8 lanes x 10 points of a group's frame (75 used)

// LDS of a grouped chunk: group starts (chunk positions; start[G] = end), the
// tile offset of each lane's ten points, scan scratch.
struct GroupLds {
  unsigned short start[kGroupMax + 2];
  int off[kGroupSlots];
  int scan[8];
};

// Exclusive scan over the 256 threads of the workgroup (sum, or max with
// identity -1 for values >= -1); scratch: 4 ints of LDS; *total receives the
// reduction over all threads.  Contains a barrier; every thread calls it.
template <bool MAX>
__device__ __forceinline__ int block_exclusive_scan(int v, int *scratch, int *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x = MAX ? max(x, y) : x + y;
  }
  if (lane == 63) scratch[wave] = x;
  int ex = __shfl_up(x, 1, 64);
  if (lane == 0) ex = MAX ? -1 : 0;
  __syncthreads();
  int pre = MAX ? -1 : 0, tot = MAX ? -1 : 0;
#pragma unroll
  for (int w = 0; w < kPushBlock / 64; ++w) {
    const int s = scratch[w];
    if (w < wave) pre = MAX ? max(pre, s) : pre + s;
    tot = MAX ? max(tot, s) : tot + s;
  }
  *total = tot;
  return MAX ? max(pre, ex) : pre + ex;
}

// Tile offset (relative to the frame origin) of point u of the 10 that lane
// k of a group holds after the reduction.  Lane k holds, for u = 0..9, pair
// p = u + 10 ((k >> 1) & 1) + 20 (k & 1), member (k >> 2) & 1 (0: first,
// 1: second) of the pairs that the first level sums:
//   p 0..11   J2 at (a = p mod 4, x3 node a3 = p / 4), x2 half point 0 | 1
//   p 12..23  J3 at (a, x2 node a2), x3 half point 0 | 1
//   p 24..32  J1 at (a = q mod 3, a2 = q / 3), x3 node 0 | 2
//   p 33..35  J1 at (a, x3 node 1), x2 node 0 | 2
//   p 36..38  J1 at (a, 1, 1) | nothing
// (x1: J1 half points, J2 and J3 nodes, from the frame's first x1 point).
__device__ __forceinline__ int group_slot_offset(int slot, int T1, int T2, int tn) {
  const int k = slot / 10, u = slot - 10 * k;
  const int p = u + 10 * ((k >> 1) & 1) + 20 * (k & 1), h = (k >> 2) & 1;
  const int T12 = T1 * T2;
  if (p < 12) return tn + (p & 3) + T1 * h + T12 * (p >> 2);
  if (p < 24) return 2 * tn + ((p - 12) & 3) + T1 * ((p - 12) >> 2) + T12 * h;
  if (p < 33) return (p - 24) % 3 + T1 * ((p - 24) / 3) + T12 * (2 * h);
  if (p < 36) return (p - 33) + T1 * (2 * h) + T12;
  if (p < 39 && h == 0) return (p - 36) + T1 + T12;
  return 0;  // padding: its value is zero
}

// Cut the runs of equal cells of the chunk's P <= 8 * 256 particles (from
// array index chunk0) into groups of at most 8 and store their starts (chunk
// positions, one thread per K = ceil(P / 256) consecutive positions) and the
// lanes' point offsets in *gl.  Returns the number of groups (the table is
// complete only when it is at most kGroupMax).  Contains barriers; every
// thread calls it.
template <typename Real>
__device__ __forceinline__ int build_groups(const Particles<Real> &p, long long chunk0, int P, int T1, int T2,
                                            int tn, GroupLds *gl) {
  const int tid = threadIdx.x;
  const int K = (P + kPushBlock - 1) / kPushBlock;
  const int pos0 = tid * K;
  int prev = INT_MIN;  // no cell has this value (dead particles are -1)
  if (pos0 > 0 && pos0 - 1 < P) prev = p.cell[chunk0 + pos0 - 1];
  int cl[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) cl[j] = (j < K && pos0 + j < P) ? p.cell[chunk0 + pos0 + j] : INT_MIN;
  // last run start among this thread's positions, then the one before them
  int last = -1;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < K && pos0 + j < P && cl[j] != (j ? cl[j - 1] : prev)) last = pos0 + j;
  int tot = 0;
  int rs = block_exclusive_scan<true>(last, gl->scan, &tot);
  // group starts: run starts and every eighth position inside a run
  int cnt = 0;
  unsigned gm = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < K && pos0 + j < P) {
      if (cl[j] != (j ? cl[j - 1] : prev)) rs = pos0 + j;
      if (((pos0 + j - rs) & 7) == 0) {
        gm |= 1u << j;
        ++cnt;
      }
    }
  int G = 0;
  int at = block_exclusive_scan<false>(cnt, gl->scan + 4, &G);
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if ((gm >> j) & 1u) {
      if (at < kGroupMax) gl->start[at] = (unsigned short)(pos0 + j);
      ++at;
    }
  if (tid == 0 && G <= kGroupMax) gl->start[G] = (unsigned short)(P > 0 ? P : 0);
  if (tid < kGroupSlots) gl->off[tid] = group_slot_offset(tid, T1, T2, tn);
  __syncthreads();
  return G;
}

// Group deposit (every lane of the wavefront calls it, in a grouped chunk):
// sums the frame-fitting particles of each 8-lane group and adds the totals
// to the LDS tile.  The first level pairs points whose values differ in one
// factor (a half-point index or a node), so each lane forms the member it
// keeps and the member it sends directly and sums them in one DPP add.
// Returns whether this lane's particle still has to be deposited (by the
// rounds, then directly).
template <typename Real>
__device__ __forceinline__ bool deposit_groups(bool active, const Moved<Real> &m, const PushParams<Real> &q,
                                               const Sink<Real> &sk, const int *goff) {
  const int lane = threadIdx.x & 63;
  const bool fits = active && m.base[0] == -1 && m.base[1] == -1 && m.base[2] == -1 && m.DS[1][3] == Real(0) &&
                    m.DS[2][3] == Real(0);
  // frame origin (cell - 1 on every axis) as a tile index, from the group's
  // first lane (its particle is the run's first; dead runs give -1)
  int fb = -1;
  if (active) fb = (m.c[0] - 1 - sk.t1) + sk.T1 * ((m.c[1] - 1 - sk.t2) + sk.T2 * (m.c[2] - 1 - sk.t3));
  fb = __builtin_amdgcn_ds_swizzle(fb, 0x18);  // lane & ~7 within each 32-lane half

  const Real z = fits ? Real(1) : Real(0);
  Real c1[3], F2[2], F3[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) c1[a] = z * q.f1 * m.cum[0][a];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    F2[h] = z * q.f2 * m.cum[1][h];
    F3[h] = z * q.f3 * m.cum[2][h];
  }
  Real P2[3], Q2[3], P3[3], Q3[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P2[k] = m.S0[1][k] + Real(0.5) * m.DS[1][k];
    Q2[k] = Real(0.5) * m.S0[1][k] + Real(1.0 / 3.0) * m.DS[1][k];
    P3[k] = m.S0[2][k] + Real(0.5) * m.DS[2][k];
    Q3[k] = Real(0.5) * m.S0[2][k] + Real(1.0 / 3.0) * m.DS[2][k];
  }
  // first level, over the row half-mirror (lane k <-> 7 - k of each group):
  // lanes 0..3 keep the first members, lanes 4..7 the second
  const bool up = (lane & 4) != 0;
  auto hm = [](Real x) { return mirror8(x); };
  Real r[39];
  {
    const Real fk = up ? F2[1] : F2[0], fs = up ? F2[0] : F2[1];
    const Real gk = up ? F3[1] : F3[0], gs = up ? F3[0] : F3[1];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const Real w2 = m.S0[0][a] * P3[k] + m.DS[0][a] * Q3[k];
        r[a + 4 * k] = fk * w2 + hm(fs * w2);
        const Real w3 = m.S0[0][a] * P2[k] + m.DS[0][a] * Q2[k];
        r[12 + a + 4 * k] = gk * w3 + hm(gs * w3);
      }
    }
  }
  {
    const Real Pk = up ? P3[2] : P3[0], Qk = up ? Q3[2] : Q3[0];
    const Real Ps = up ? P3[0] : P3[2], Qs = up ? Q3[0] : Q3[2];
#pragma unroll
    for (int a2 = 0; a2 < 3; ++a2) {
      const Real wk = m.S0[1][a2] * Pk + m.DS[1][a2] * Qk, ws = m.S0[1][a2] * Ps + m.DS[1][a2] * Qs;
#pragma unroll
      for (int a = 0; a < 3; ++a) r[24 + a + 3 * a2] = c1[a] * wk + hm(c1[a] * ws);
    }
    const Real Sk = up ? m.S0[1][2] : m.S0[1][0], Dk = up ? m.DS[1][2] : m.DS[1][0];
    const Real Ss = up ? m.S0[1][0] : m.S0[1][2], Ds = up ? m.DS[1][0] : m.DS[1][2];
    const Real wk = Sk * P3[1] + Dk * Q3[1], ws = Ss * P3[1] + Ds * Q3[1];
    const Real w11 = m.S0[1][1] * P3[1] + m.DS[1][1] * Q3[1];
    const Real w11k = up ? Real(0) : w11, w11s = up ? w11 : Real(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r[33 + a] = c1[a] * wk + hm(c1[a] * ws);
      r[36 + a] = c1[a] * w11k + hm(c1[a] * w11s);
    }
  }
  // second and third levels: lane ^ 1 (39 -> 20 values), lane ^ 2 (-> 10)
  int off = 0;
  rs_level<Real, 39, 1>(r, lane, off);
  rs_level<Real, 20, 2>(r, lane, off);
  if (fb >= 0) {
    double *base = sk.tile_d + fb;
    // all ten offsets are read before the first add: the adds could alias
    // the table, so a read placed after an add would wait for it
    const int *lo = goff + (lane & 7) * 10;
    int o[10];
#pragma unroll
    for (int u = 0; u < 10; ++u) o[u] = lo[u];
#pragma unroll
    for (int u = 0; u < 10; ++u) lds_add(base + o[u], (double)r[u]);
  }
  return active && !fits;
}

// One workgroup's share of the particle phase: the particles at array
// indices [chunk0, chunk1), K = ceil((chunk1 - chunk0) / 256) per thread.
// tile_raw: TILE bytes of LDS, box: kChunkBoxInts ints of LDS; *mybox receives
// the chunk's deposit box.  With W = 4 (tile-sorted 3D species) gl is the LDS
// of the cell groups: a chunk of at most 2048 particles whose current fits
// the LDS tile in FP64 and whose runs of equal cells make at most 32 (K + 1)
// groups of <= 8 particles is walked group by group (ceil(groups / 32)
// iterations), others 256 particles per iteration in array order.  ROUNDS
// = false (species whose cells hold long runs): lanes that leave the group
// sums deposit directly, without the wavefront rounds, whose code alone
// costs the loop registers (SGPR spills reloaded every iteration).
template <typename Real, int DIM, int W = 2, int TILE = kTileBytes, bool ROUNDS = true>
__device__ __forceinline__ void push_chunk(const Geo &g, const Fields<Real> &f, const HalfB<Real> &Bh,
                                           const Particles<Real> &p, const PushParams<Real> &q, long long chunk0,
                                           long long chunk1, JBox *mybox, int *err, unsigned char *tile_raw,
                                           int *box, GroupLds *gl = nullptr) {
  Real *tile = reinterpret_cast<Real *>(tile_raw);
  if (chunk1 > p.n) chunk1 = p.n;
  if (chunk0 > chunk1) chunk0 = chunk1;
  const int P = (int)(chunk1 - chunk0);
  const int K = (P + kPushBlock - 1) / kPushBlock;
  const int tid = threadIdx.x;

  // wave priorities by phase: the box and staging passes (between
  // barriers) 2, the particle loop 0, the flush 1
  __builtin_amdgcn_s_setprio(2);
  // ---- chunk bounding box (window x1, x2, x3) of the particles' old cells
  if (tid == 0) {
    box[0] = box[2] = box[4] = INT_MAX;
    box[1] = box[3] = box[5] = INT_MIN;
  }
  __syncthreads();
  {
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
    // the cells of up to 8 particles per thread are loaded together, so their
    // latencies overlap
    for (int k0 = 0; k0 < K; k0 += 8) {
      int cells[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const long long i = chunk0 + (long long)(k0 + j) * kPushBlock + tid;
        cells[j] = (k0 + j < K && i < chunk1) ? p.cell[i] : -1;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int packed = cells[j];
        if (packed < 0) continue;
        int s1, c2, c3;
        unpack_cell(g, packed, s1, c2, c3);
        int c1 = s1 - g.ws_mod;
        if (c1 < 0) c1 += g.n1;
        const int cc[3] = {c1, c2, c3};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          mn[d] = min(mn[d], cc[d]);
          mx[d] = max(mx[d], cc[d]);
        }
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      mn[d] = wave_min(mn[d]);
      mx[d] = wave_max(mx[d]);
    }
    if ((tid & 63) == 0 && mn[0] != INT_MAX) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        atomicMin(&box[2 * d], mn[d]);
        atomicMax(&box[2 * d + 1], mx[d]);
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    // deposits of this chunk land within its old cells +- 2; empty chunks
    // write an empty box
    int lo[3] = {box[0] - 2, box[2] - 2, DIM == 3 ? box[4] - 2 : 0};
    int hi[3] = {box[1] + 2, box[3] + 2, DIM == 3 ? box[5] + 2 : 0};
    const int nn[3] = {g.n1, g.n2, g.n3};
    if (box[0] == INT_MAX) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = INT_MAX;
        hi[d] = -INT_MAX;
      }
    } else {
      if (g.window) {
        lo[0] = max(lo[0], 0);
        hi[0] = min(hi[0], g.n1 - 1);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (lo[d] < 0 || hi[d] >= nn[d]) {
          lo[d] = 0;
          hi[d] = nn[d] - 1;
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      mybox->lo[d] = lo[d];
      mybox->hi[d] = hi[d];
    }
    // dividers for the tile's x1 and x2 extents (old cells +- 2)
    if (box[0] != INT_MAX) {
      const FastDiv a = make_fastdiv((unsigned)(box[1] - box[0] + 5)), b = make_fastdiv((unsigned)(box[3] - box[2] + 5));
      box[6] = (int)a.m;
      box[7] = a.L;
      box[8] = (int)b.m;
      box[9] = b.L;
    }
  }
  __syncthreads();
  Sink<Real> sk;
  sk.g = g;
  sk.J[0] = f.J1;
  sk.J[1] = f.J2;
  sk.J[2] = f.J3;
  sk.tile = nullptr;
  sk.tile_d = nullptr;
  sk.t1 = box[0] - 2;
  sk.t2 = box[2] - 2;
  sk.t3 = DIM == 3 ? box[4] - 2 : 0;
  sk.T1 = sk.T2 = sk.T3 = 1;
  sk.tn = 0;
  if (box[0] != INT_MAX) {
    const long long T1 = (long long)box[1] - box[0] + 5, T2 = (long long)box[3] - box[2] + 5;
    const long long T3 = DIM == 3 ? (long long)box[5] - box[4] + 5 : 1;
    // FP32 runs: current in FP64 words when they fit
    const bool j64 = sizeof(Real) == 4 && 12 * T1 * T2 * T3 * (long long)sizeof(Real) <= TILE;
    if (j64 || 9 * T1 * T2 * T3 * (long long)sizeof(Real) <= TILE) {
      sk.T1 = (int)T1;
      sk.T2 = (int)T2;
      sk.T3 = (int)T3;
      sk.tn = (int)(T1 * T2 * T3);
      sk.tile = tile;
      // FP64 current words: the tile's own in an FP64 run
      if (j64 || sizeof(Real) == 8) sk.tile_d = reinterpret_cast<double *>(tile_raw);
      Real *fE = tile + (j64 ? 6 : 3) * sk.tn;
      // J part cleared; E and B^n staged for the gather (zero outside the
      // window), one tile cell per thread and pass
      const int tn = sk.tn;
      const FastDiv d1{(unsigned)box[6], box[7]}, d2{(unsigned)box[8], box[9]};
      for (int r = tid; r < tn; r += kPushBlock) {
        const int q1 = (int)fdiv(d1, (unsigned)r), q2 = (int)fdiv(d2, (unsigned)q1);
        const int a1 = r - q1 * sk.T1, a2 = q1 - q2 * sk.T2;
        // the gather reads cells c - 2 .. c + 1 of each axis, so the box's
        // last layer on each axis (old cells + 2) holds current only
        const bool used = a1 < sk.T1 - 1 && a2 < sk.T2 - 1 && (DIM == 2 || q2 < sk.T3 - 1);
        const int col = used ? col_of(g, sk.t1 + a1) : -1;
        Real v[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
        if (col >= 0) {
          const unsigned id =
              (unsigned)g.n1 * (unsigned)(wrap_near(sk.t2 + a2, g.n2) + g.n2 * wrap_near(sk.t3 + q2, g.n3)) +
              (unsigned)col;
          v[0] = ld32(f.E1, id);
          v[1] = ld32(f.E2, id);
          v[2] = ld32(f.E3, id);
          v[3] = Real(0.5) * (ld32(f.B1, id) + ld32(Bh.B1, id));
          v[4] = Real(0.5) * (ld32(f.B2, id) + ld32(Bh.B2, id));
          v[5] = Real(0.5) * (ld32(f.B3, id) + ld32(Bh.B3, id));
        }
        if (j64) {
#pragma unroll
          for (int k = 0; k < 3; ++k) sk.tile_d[k * tn + r] = 0.0;
        } else {
#pragma unroll
          for (int k = 0; k < 3; ++k) tile[k * tn + r] = Real(0);
        }
        if (used) {
#pragma unroll
          for (int k = 0; k < 6; ++k) fE[k * tn + r] = v[k];
        }
      }
    }
  }
  __syncthreads();
  const bool lds_fields = sk.tile != nullptr;
  // cell groups: the chunk's runs of equal cells in pieces of <= 8
  int nit = K, G = 0;
  bool grouped = false;
  if constexpr (W == 4 && DIM == 3) {
    if (lds_fields) {
      if (K <= 8) G = build_groups<Real>(p, chunk0, P, sk.T1, sk.T2, sk.tn, gl);
      grouped = sk.tile_d != nullptr && K <= 8 && G > 0 && G <= 32 * (K + 1);
      if (grouped) nit = (G + 31) / 32;
    }
  }
  // array index of this thread's particle in iteration it (-1: none)
  auto index_of = [&](int it) -> long long {
    if constexpr (W == 4 && DIM == 3) {
      if (grouped) {
        const int gi = it * 32 + (tid >> 3);
        if (gi >= G) return -1;
        const int s0 = gl->start[gi], e0 = gl->start[gi + 1], k8 = tid & 7;
        return s0 + k8 < e0 ? chunk0 + s0 + k8 : -1;
      }
    }
    const long long i = chunk0 + (long long)it * kPushBlock + tid;
    return i < chunk1 ? i : -1;
  };

  __builtin_amdgcn_s_setprio(0);
  // ---- gather, push, move and deposit, K particles per thread (grouped:
  // one per group member); the next particle's state is loaded while the
  // current one is pushed
  int nx_cell = -1;
  Real nx_o[3] = {Real(0), Real(0), Real(0)}, nx_u[3] = {Real(0), Real(0), Real(0)};
  auto load_state = [&](long long j) {
    nx_cell = -1;
    if (j >= 0 && j < p.n) {
      const unsigned jj = (unsigned)j;
      nx_cell = el32(p.cell, jj);
      nx_o[0] = el32(p.o1, jj);
      nx_o[1] = el32(p.o2, jj);
      if (DIM == 3) nx_o[2] = el32(p.o3, jj);
      nx_u[0] = el32(p.u1, jj);
      nx_u[1] = el32(p.u2, jj);
      nx_u[2] = el32(p.u3, jj);
    }
  };
  long long nx_i = index_of(0);
  load_state(nx_i);
  for (int k = 0; k < nit; ++k) {
    const long long i = nx_i;
    const int packed = nx_cell;
    const Real o[3] = {nx_o[0], nx_o[1], nx_o[2]}, u0[3] = {nx_u[0], nx_u[1], nx_u[2]};
    if (k + 1 < nit) {
      nx_i = index_of(k + 1);
      load_state(nx_i);
    }
    const bool active = packed >= 0;
    Moved<Real> m;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      m.c[d] = 0;
      m.base[d] = -1;
#pragma unroll
      for (int a = 0; a < 4; ++a) m.S0[d][a] = m.DS[d][a] = m.cum[d][a] = Real(0);
    }
    m.jz = 0;
    if (active) {
      int s1, c2, c3;
      unpack_cell(g, packed, s1, c2, c3);
      int c1 = s1 - g.ws_mod;
      if (c1 < 0) c1 += g.n1;
      m.c[0] = c1;
      m.c[1] = c2;
      m.c[2] = c3;

      Real E1, E2, E3, B1, B2, B3;
      Stagger<Real> st;
      int bH[3];
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        qw(o[d], st.wN[d]);
        bH[d] = qw_half(m.c[d], o[d], st.wH[d]);
      }
      if (lds_fields) {
        StaggerL sl;
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
          sl.x1[k2] = c1 - 2 + k2 - sk.t1;
          sl.x2[k2] = sk.T1 * (c2 - 2 + k2 - sk.t2);
          sl.x3[k2] = sk.T1 * sk.T2 * (c3 - 2 + k2 - sk.t3);
        }
        sl.h1lo = bH[0] < c1;
        sl.h2lo = bH[1] < c2;
        sl.h3lo = DIM == 3 && bH[2] < c3;
        // E and B follow the current: 3 words per cell in its own precision,
        // 6 when an FP32 run holds it in FP64
        const Real *ft = tile + ((sizeof(Real) == 4 && sk.tile_d) ? 6 : 3) * sk.tn;
        E1 = interp_lds<Real, DIM, true, false, false>(sl, st.wN, st.wH, ft);
        E2 = interp_lds<Real, DIM, false, true, false>(sl, st.wN, st.wH, ft + sk.tn);
        E3 = interp_lds<Real, DIM, false, false, true>(sl, st.wN, st.wH, ft + 2 * sk.tn);
        B1 = interp_lds<Real, DIM, false, true, true>(sl, st.wN, st.wH, ft + 3 * sk.tn);
        B2 = interp_lds<Real, DIM, true, false, true>(sl, st.wN, st.wH, ft + 4 * sk.tn);
        B3 = interp_lds<Real, DIM, true, true, false>(sl, st.wN, st.wH, ft + 5 * sk.tn);
      } else {
      {
        // window cells c-2 .. c+1 cover both stencils (half: bH-1 .. bH+1, bH in {c-1, c})
        int cx[4];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) cx[k2] = col_near(g, c1 - 2 + k2);
        const bool hlo = bH[0] < c1;
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) {
          const int cn = cx[a2 + 1], ch = hlo ? cx[a2] : cx[a2 + 1];
          st.colN[a2] = cn < 0 ? 0u : (unsigned)cn;
          st.colH[a2] = ch < 0 ? 0u : (unsigned)ch;
          if (cn < 0) st.wN[0][a2] = Real(0);
          if (ch < 0) st.wH[0][a2] = Real(0);
        }
        unsigned r2x[4];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) r2x[k2] = (unsigned)g.n1 * (unsigned)wrap_near(c2 - 2 + k2, g.n2);
        const bool h2lo = bH[1] < c2;
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) {
          st.rowN2[a2] = r2x[a2 + 1];
          st.rowH2[a2] = h2lo ? r2x[a2] : r2x[a2 + 1];
        }
        if (DIM == 3) {
          unsigned r3x[4];
#pragma unroll
          for (int k2 = 0; k2 < 4; ++k2)
            r3x[k2] = (unsigned)g.n1 * (unsigned)g.n2 * (unsigned)wrap_near(c3 - 2 + k2, g.n3);
          const bool h3lo = bH[2] < c3;
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2) {
            st.rowN3[a2] = r3x[a2 + 1];
            st.rowH3[a2] = h3lo ? r3x[a2] : r3x[a2 + 1];
          }
        }
      }
      E1 = interp<Real, DIM, true, false, false, false>(st, f.E1, nullptr);
      E2 = interp<Real, DIM, false, true, false, false>(st, f.E2, nullptr);
      E3 = interp<Real, DIM, false, false, true, false>(st, f.E3, nullptr);
      B1 = interp<Real, DIM, false, true, true, true>(st, f.B1, Bh.B1);
      B2 = interp<Real, DIM, true, false, true, true>(st, f.B2, Bh.B2);
      B3 = interp<Real, DIM, true, true, false, true>(st, f.B3, Bh.B3);

      }

      // relativistic Boris push
      const Real a = q.half_qmdt;
      const Real um1 = u0[0] + a * E1, um2 = u0[1] + a * E2, um3 = u0[2] + a * E3;
      const Real ag = a * push_rsqrt(Real(1) + um1 * um1 + um2 * um2 + um3 * um3);
      const Real t1 = ag * B1, t2 = ag * B2, t3 = ag * B3;
      const Real t2s = t1 * t1 + t2 * t2 + t3 * t3;
      const Real f2 = Real(2) * push_rcp(Real(1) + t2s);
      const Real s1v = f2 * t1, s2v = f2 * t2, s3v = f2 * t3;
      const Real up1 = um1 + (um2 * t3 - um3 * t2);
      const Real up2 = um2 + (um3 * t1 - um1 * t3);
      const Real up3 = um3 + (um1 * t2 - um2 * t1);
      const Real un1 = um1 + (up2 * s3v - up3 * s2v) + a * E1;
      const Real un2 = um2 + (up3 * s1v - up1 * s3v) + a * E2;
      const Real un3 = um3 + (up1 * s2v - up2 * s1v) + a * E3;
      const Real ig = push_rsqrt(Real(1) + un1 * un1 + un2 * un2 + un3 * un3);
      if (!(un1 == un1) || !(un2 == un2) || !(un3 == un3)) atomicOr(err, 2);

      // x^{n+1} = x^n + dt u / gamma, in cell units, as cell + offset
      const Real un[3] = {un1, un2, un3};
      int sh[3] = {0, 0, 0};
      Real on[3] = {o[0], o[1], o[2]};
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const Real dlt = q.dtdx[d] * un[d] * ig;
        if (!(dlt < Real(1) && dlt > Real(-1))) atomicOr(err, 1);
        const Real v = o[d] + dlt;
        int kk = 0;
        if (v >= Real(0.5))
          kk = 1;
        else if (v < Real(-0.5))
          kk = -1;
        sh[d] = kk;
        on[d] = v - Real(kk);
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d) m.base[d] = esirkepov_1d(o[d], sh[d], on[d], m.S0[d], m.DS[d], m.cum[d]);
      if (DIM == 2) {
        // the out-of-plane direction carries the time-averaged shape weight
        m.jz = q.fv * un3 * ig;
      }

      // store the new state
      const int n1c = c1 + sh[0];
      bool alive = true;
      if (g.window) {
        const int after = n1c - q.shift;  // window cell after this step's shift
        if (after < 2 || after > g.n1 - 3) alive = false;
      }
      const unsigned ii = (unsigned)i;
      if (!alive) {
        el32(p.cell, ii) = -1;
      } else {
        const int ns1 = col_of(g, n1c);
        const int ns2 = wrap_near(c2 + sh[1], g.n2);
        const int ns3 = DIM == 3 ? wrap_near(c3 + sh[2], g.n3) : 0;
        el32(p.cell, ii) = ns1 + g.n1 * (ns2 + g.n2 * ns3);
        el32(p.o1, ii) = on[0];
        el32(p.o2, ii) = on[1];
        if (DIM == 3) el32(p.o3, ii) = on[2];
        el32(p.u1, ii) = un1;
        el32(p.u2, ii) = un2;
        el32(p.u3, ii) = un3;
      }
    }
    bool rest = active;
    if constexpr (W == 4 && DIM == 3) {
      if (grouped) rest = deposit_groups<Real>(active, m, q, sk, gl->off);
    }
    if constexpr (W == 4 && DIM == 3 && !ROUNDS) {
      if (rest) deposit_direct<Real, DIM>(m, q, sk);
    } else {
      if (deposit_wave<Real, DIM, W>(rest, m, q, sk)) deposit_direct<Real, DIM>(m, q, sk);
    }
  }

  __builtin_amdgcn_s_setprio(1);
  // ---- flush the tile to HBM: one atomic per non-zero point
  if (sk.tile) {
    __syncthreads();
    const FastDiv d1{(unsigned)box[6], box[7]}, d2{(unsigned)box[8], box[9]};
    for (int r = tid; r < sk.tn; r += kPushBlock) {
      Real v[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) v[k] = sk.tile_d ? (Real)sk.tile_d[k * sk.tn + r] : tile[k * sk.tn + r];
      if (v[0] == Real(0) && v[1] == Real(0) && v[2] == Real(0)) continue;
      const int q1 = (int)fdiv(d1, (unsigned)r), q2 = (int)fdiv(d2, (unsigned)q1);
      const int col = col_near(g, sk.t1 + r - q1 * sk.T1);
      if (col < 0) continue;
      const unsigned id = (unsigned)g.n1 * (unsigned)(wrap_near(sk.t2 + q1 - q2 * sk.T2, g.n2) +
                                                       g.n2 * wrap_near(sk.t3 + q2, g.n3)) + (unsigned)col;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (v[k] != Real(0)) atomicAdd(&el32(sk.J[k], id), v[k]);
    }
  }
}


}  // namespace relpic
