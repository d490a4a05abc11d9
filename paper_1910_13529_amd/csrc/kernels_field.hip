// Maxwell field advance on the Yee lattice (Eq. 1 with the operators of
// Eq. 14 and, along x1, the customized 2M-point operator of App. C), and the
// J1 current correction of the customized solver (Sec. 3).
//
// B is kept at half-integer times in two buffers, so one step is
//   B^{n+1/2} = B^{n-1/2} - dt d+ x E^n                   (k_curl_e)
//   E^{n+1}   = E^n + dt d- x B^{n+1/2}                    (k_curl_b)
//   E^{n+1}  -= dt J^{n+1/2} inside the deposit's box       (k_add_j)
// which is the leapfrog of the split B half steps; the gather takes
// B^n = (B^{n-1/2} + B^{n+1/2}) / 2.  Each workgroup takes a 256-cell x1
// segment and marches through consecutive rows (2D: x2) or planes (3D: x3),
// staging each row and its 2M-cell halo in LDS for the axial stencil;
// workgroups are renumbered so that each XCD sweeps a contiguous band of
// rows (neighbouring rows share its L2).
#include "field_tiles.h"
#include "xlane.h"

namespace relpic {

// 2D: each workgroup takes one 256-cell x1 segment and marches through
// `rows` consecutive x2 rows (curl_e_rows / curl_b_rows); rows shrinks on
// small grids so that the launch still has about 2048 workgroups.
constexpr int kMaxRows = 8;

__host__ inline int rows_per_tile(const Geo &g) {
  const long long nseg = (g.n1 + kSeg - 1) / kSeg;
  const long long r = nseg * g.n2 / 2048;
  return (int)(r < 1 ? 1 : (r > kMaxRows ? kMaxRows : r));
}

__device__ __forceinline__ bool rows_of(const Geo &g, int nseg, int rows, int &l0, int &r0, int &r1) {
  const int nr = (g.n2 + rows - 1) / rows;
  const long long nb = (long long)nseg * nr;
  const long long per = (nb + kNumXcd - 1) / kNumXcd;
  const long long bid = blockIdx.x;
  const long long lin = (bid % kNumXcd) * per + bid / kNumXcd;
  if (lin >= nb) return false;
  l0 = (int)(lin % nseg) * kSeg;
  r0 = (int)(lin / nseg) * rows;
  r1 = min(r0 + rows, g.n2);
  return true;
}

__host__ inline unsigned rows_blocks(const Geo &g, int rows) {
  const long long nb = (long long)((g.n1 + kSeg - 1) / kSeg) * ((g.n2 + rows - 1) / rows);
  return (unsigned)((nb + kNumXcd - 1) / kNumXcd * kNumXcd);
}

template <typename Real, int MM>
__global__ __launch_bounds__(kSeg) void k_curl_e_2d(Geo g, Fields<Real> f, const Real *Bin1, const Real *Bin2,
                                                    const Real *Bin3, Real *Bout1, Real *Bout2, Real *Bout3,
                                                    Axial<Real> ax, Real h2, int rows) {
  __shared__ Real sE2[stage_pitch<kSeg>()], sE3[stage_pitch<kSeg>()];
  int l0, r0, r1;
  if (!rows_of(g, (g.n1 + kSeg - 1) / kSeg, rows, l0, r0, r1)) return;
  curl_e_rows<Real, MM, kSeg>(g, f.E1, f.E2, f.E3, Bin1, Bin2, Bin3, Bout1, Bout2, Bout3, ax, h2, l0, r0, r1, sE2,
                              sE3);
}

template <typename Real, int MM>
__global__ __launch_bounds__(kSeg) void k_curl_b_2d(Geo g, Fields<Real> f, Axial<Real> ax, Real e2, int rows) {
  __shared__ Real sB2[stage_pitch<kSeg>()], sB3[stage_pitch<kSeg>()];
  int l0, r0, r1;
  if (!rows_of(g, (g.n1 + kSeg - 1) / kSeg, rows, l0, r0, r1)) return;
  curl_b_rows<Real, MM, kSeg>(g, f.E1, f.E2, f.E3, f.B1, f.B2, f.B3, ax, e2, l0, r0, r1, sB2, sB3);
}

// 3D: each workgroup takes one 256-cell x1 segment of one x2 row and marches
// through kPlanes consecutive x3 planes, carrying the x3 neighbour it has
// already loaded in registers (E at i3 + 1 becomes the next plane's own E for
// the B update; B at i3 becomes the next plane's i3 - 1 for the E update), so
// every array is read from HBM once per launch.
constexpr int kPlanes = 8;

__device__ __forceinline__ bool column_of(const Geo &g, int nseg, int &l0, int &i2, int &z0, int &z1) {
  const int nz = (g.n3 + kPlanes - 1) / kPlanes;
  const long long nb = (long long)nseg * g.n2 * nz;
  const long long per = (nb + kNumXcd - 1) / kNumXcd;
  const long long bid = blockIdx.x;
  const long long lin = (bid % kNumXcd) * per + bid / kNumXcd;
  if (lin >= nb) return false;
  const int seg = (int)(lin % nseg);
  const long long r = lin / nseg;
  i2 = (int)(r % g.n2);
  const int zc = (int)(r / g.n2);
  l0 = seg * kSeg;
  z0 = zc * kPlanes;
  z1 = min(z0 + kPlanes, g.n3);
  return true;
}

__host__ inline unsigned column_blocks(const Geo &g) {
  const long long nseg = (g.n1 + kSeg - 1) / kSeg;
  const long long nb = nseg * g.n2 * ((g.n3 + kPlanes - 1) / kPlanes);
  const long long per = (nb + kNumXcd - 1) / kNumXcd;
  return (unsigned)(per * kNumXcd);
}

// Bout = Bin - curl+ E, marching over x3 (coefficients as in curl_e_tile).
// Every global operand of plane i3 + 1 (the staged row, the own cell's Bin,
// its x3 and x2 neighbours' E) is loaded while plane i3 is computed.
template <typename Real, int MM>
__global__ __launch_bounds__(kSeg) void k_curl_e_col(Geo g, Fields<Real> f, const Real *Bin1, const Real *Bin2,
                                                     const Real *Bin3, Real *Bout1, Real *Bout2, Real *Bout3,
                                                     Axial<Real> ax, Real h2, Real h3) {
  __shared__ Real sE2[stage_pitch<kSeg>()], sE3[stage_pitch<kSeg>()];
  int l0, i2, z0, z1;
  if (!column_of(g, (g.n1 + kSeg - 1) / kSeg, l0, i2, z0, z1)) return;
  const int M = MM > 0 ? MM : ax.M;
  const int l1 = l0 + threadIdx.x;
  const bool live = l1 < g.n1;
  const int s1 = live ? col_near(g, l1) : -1;
  const bool own = live && s1 >= 0;
  const long long plane = (long long)g.n1 * g.n2;
  const long long r2 = (long long)g.n1 * i2, r2p = (long long)g.n1 * wrap_near(i2 + 1, g.n2);
  const int c = threadIdx.x + M - 1;  // LDS index of cell l1
  // the staged row (cells l0 - M + 1 .. l0 + 255 + M) is at most two values
  // per thread and array
  const int ta = threadIdx.x, tb = threadIdx.x + kSeg;
  const bool hb = tb < kSeg + 2 * M;
  const int ca = col_of(g, l0 - M + 1 + ta), cb = hb ? col_of(g, l0 - M + 1 + tb) : -1;
  Real a2, a3, b2, b3;                                            // staged E2, E3
  Real e1u = 0, e2u = 0, e1r = 0, e3r = 0, q1 = 0, q2 = 0, q3 = 0;  // own cell's operands
  auto fetch = [&](int i3) {
    const long long row = r2 + plane * i3;
    a2 = ldc(f.E2, row, ca);
    a3 = ldc(f.E3, row, ca);
    b2 = ldc(f.E2, row, cb);
    b3 = ldc(f.E3, row, cb);
    if (own) {
      const long long id = row + s1, up = r2 + plane * wrap_near(i3 + 1, g.n3) + s1, id2 = r2p + plane * i3 + s1;
      e1u = f.E1[up];
      e2u = f.E2[up];
      e1r = f.E1[id2];
      e3r = f.E3[id2];
      q1 = Bin1[id];
      q2 = Bin2[id];
      q3 = Bin3[id];
    }
  };
  Real e1 = own ? f.E1[r2 + plane * z0 + s1] : Real(0);
  fetch(z0);
  for (int i3 = z0; i3 < z1; ++i3) {
    sE2[ta] = a2;
    sE3[ta] = a3;
    if (hb) {
      sE2[tb] = b2;
      sE3[tb] = b3;
    }
    const Real ce1u = e1u, ce2u = e2u, ce1r = e1r, ce3r = e3r, cq1 = q1, cq2 = q2, cq3 = q3;
    __syncthreads();
    if (i3 + 1 < z1) fetch(i3 + 1);
    if (own) {
      const long long id = r2 + plane * i3 + s1;
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
      const Real e2 = sE2[c], e3 = sE3[c];
      const Real d2E3 = h2 * (ce3r - e3);
      const Real d2E1 = h2 * (ce1r - e1);
      const Real d3E2 = h3 * (ce2u - e2);
      const Real d3E1 = h3 * (ce1u - e1);
      Bout1[id] = cq1 - (d2E3 - d3E2);
      Bout2[id] = cq2 - (d3E1 - d1E3);
      Bout3[id] = cq3 - (d1E2 - d2E1);
      e1 = ce1u;
    }
    __syncthreads();
  }
}

// E += curl- B, marching over x3 (coefficients as in curl_b_tile), operands
// of the next plane loaded while the current one is computed
template <typename Real, int MM>
__global__ __launch_bounds__(kSeg) void k_curl_b_col(Geo g, Fields<Real> f, Axial<Real> ax, Real e2c, Real e3c) {
  __shared__ Real sB2[stage_pitch<kSeg>()], sB3[stage_pitch<kSeg>()];
  int l0, i2, z0, z1;
  if (!column_of(g, (g.n1 + kSeg - 1) / kSeg, l0, i2, z0, z1)) return;
  const int M = MM > 0 ? MM : ax.M;
  const int l1 = l0 + threadIdx.x;
  const bool live = l1 < g.n1;
  const int s1 = live ? col_near(g, l1) : -1;
  const bool own = live && s1 >= 0;
  const long long plane = (long long)g.n1 * g.n2;
  const long long r2 = (long long)g.n1 * i2, r2m = (long long)g.n1 * wrap_near(i2 - 1, g.n2);
  const int c = threadIdx.x + M;  // LDS index of cell l1
  Real b1m = Real(0), b2m = Real(0);
  if (own) {
    const long long dn = r2 + plane * wrap_near(z0 - 1, g.n3) + s1;
    b1m = f.B1[dn];
    b2m = f.B2[dn];
  }
  const int ta = threadIdx.x, tb = threadIdx.x + kSeg;
  const bool hb = tb < kSeg + 2 * M;
  const int ca = col_of(g, l0 - M + ta), cb = hb ? col_of(g, l0 - M + tb) : -1;
  Real a2, a3, b2s, b3s;                                           // staged B2, B3
  Real b1 = 0, b1r = 0, b3r = 0, x1 = 0, x2 = 0, x3 = 0;           // own cell's operands
  auto fetch = [&](int i3) {
    const long long row = r2 + plane * i3;
    a2 = ldc(f.B2, row, ca);
    a3 = ldc(f.B3, row, ca);
    b2s = ldc(f.B2, row, cb);
    b3s = ldc(f.B3, row, cb);
    if (own) {
      const long long id = row + s1, id2 = r2m + plane * i3 + s1;
      b1 = f.B1[id];
      b1r = f.B1[id2];
      b3r = f.B3[id2];
      x1 = f.E1[id];
      x2 = f.E2[id];
      x3 = f.E3[id];
    }
  };
  fetch(z0);
  for (int i3 = z0; i3 < z1; ++i3) {
    sB2[ta] = a2;
    sB3[ta] = a3;
    if (hb) {
      sB2[tb] = b2s;
      sB3[tb] = b3s;
    }
    const Real cb1 = b1, cb1r = b1r, cb3r = b3r, cx1 = x1, cx2 = x2, cx3 = x3;
    __syncthreads();
    if (i3 + 1 < z1) fetch(i3 + 1);
    if (own) {
      const long long id = r2 + plane * i3 + s1;
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
      const Real bb2 = sB2[c], bb3 = sB3[c];
      const Real d2B3 = e2c * (bb3 - cb3r);
      const Real d2B1 = e2c * (cb1 - cb1r);
      const Real d3B2 = e3c * (bb2 - b2m);
      const Real d3B1 = e3c * (cb1 - b1m);
      f.E1[id] = cx1 + (d2B3 - d3B2);
      f.E2[id] = cx2 + (d3B1 - d1B3);
      f.E3[id] = cx3 + (d1B2 - d2B1);
      b1m = cb1;
      b2m = bb2;
    }
    __syncthreads();
  }
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

// J cleared over the box of deposited current (the fused update has added
// it to E); one thread resets the box used by the next step's deposit.
template <typename Real>
__global__ __launch_bounds__(256) void k_clear_j(Geo g, Fields<Real> f, const JBox *box, int pad, JBox *next) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) {
      next->lo[d] = 0x7fffffff;
      next->hi[d] = -0x7fffffff;
    }
  }
  clear_j_box(g, f.J1, f.J2, f.J3, *box, pad, blockIdx.x * (long long)blockDim.x + threadIdx.x,
              (long long)gridDim.x * blockDim.x);
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

// The same correction one x1 line of the box at a time: a workgroup stages
// the line's J1 (box x1 range widened by 2 ng) in LDS and every output reads
// its 2 ng + 1 taps from there (same arithmetic as jcorr_box).  For boxes
// that cover much of the grid (a beam in a plasma) it replaces ~2 ng + 1
// cached global loads per cell by one.
template <typename Real>
__global__ __launch_bounds__(256) void k_jcorr_rows(Geo g, const Real *J1, Real *J1c, const Real *taps, int ng,
                                                    const JBox *box) {
  extern __shared__ __align__(16) unsigned char jc_lds[];
  Real *line = reinterpret_cast<Real *>(jc_lds);
  const JBox b = *box;
  int lo1, hi1;
  if (!box_x1(g, b, ng, lo1, hi1)) return;  // whole workgroup
  const int W = hi1 - lo1 + 1;
  const long long w2 = b.hi[1] - b.lo[1] + 1, rows = w2 * (b.hi[2] - b.lo[2] + 1);
  for (long long r = blockIdx.x; r < rows; r += gridDim.x) {
    const int i2 = b.lo[1] + (int)(r % w2), i3 = b.lo[2] + (int)(r / w2);
    const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
    // one cell past the last tap of the last output: an odd W's second
    // output of the last pair reads it (and is not stored)
    for (int t = threadIdx.x; t < W + 2 * ng + 1; t += blockDim.x) line[t] = ldc(J1, row, col_of(g, lo1 - ng + t));
    __syncthreads();
    // two neighbouring outputs j, j + 1 per thread: per tap m the pair reads
    // c[j - m] and c[j + 1 + m] and takes c[j + m], c[j + 1 - m] from the
    // previous tap, so each LDS word read serves both outputs
    for (int t = 2 * threadIdx.x; t < W; t += 2 * blockDim.x) {
      const Real *c = line + ng + t;
      Real a0 = taps[0] * c[0], a1 = taps[0] * c[1];
      Real lprev = c[0], rprev = c[1];
#pragma unroll 4
      for (int m = 1; m <= ng; ++m) {
        const Real l = c[-m], r = c[1 + m];
        const Real tm = taps[m];
        a0 += tm * (l + rprev);
        a1 += tm * (lprev + r);
        lprev = l;
        rprev = r;
      }
      J1c[row + col_of(g, lo1 + t)] = a0;
      if (t + 1 < W) J1c[row + col_of(g, lo1 + t + 1)] = a1;
    }
    __syncthreads();
  }
}

// Current filter (the 5-pass smoothing with which Secs. 2.2-3 quote the
// filtered self-force): on each x1 line of the box, npass passes of the binomial
// (1/4, 1/2, 1/4) and then one compensating pass (ca, cb, ca), in place.  A
// pass treats the line as zero beyond a moving window's ends and wraps on a
// periodic line.  The input is the box's x1 range widened by in_pad (cells
// outside it are taken as zero whatever the buffer holds there, e.g. stale
// J1c); the output, written back, is that range widened by npass + 1, which
// holds the whole support of the result.  One workgroup per (line,
// component): the line is staged in LDS, and a pass reads every cell's three
// operands into registers, waits, and writes the results back.
constexpr int kFilterPer = kFilterMaxLine / 256;

template <typename Real>
__global__ __launch_bounds__(256) void k_filter_rows(Geo g, Real *A0, Real *A1, Real *A2, const JBox *box,
                                                     int in_pad, int npass, Real ca, Real cb) {
  extern __shared__ __align__(16) unsigned char fl_lds[];
  Real *line = reinterpret_cast<Real *>(fl_lds);
  JBox b;
  if (box) {
    b = *box;
  } else {
    b.lo[0] = b.lo[1] = b.lo[2] = 0;
    b.hi[0] = g.n1 - 1;
    b.hi[1] = g.n2 - 1;
    b.hi[2] = g.n3 - 1;
  }
  int va, vb, oa, ob;
  if (!box_x1(g, b, in_pad, va, vb)) return;  // whole workgroup
  box_x1(g, b, in_pad + npass + 1, oa, ob);
  const int L = ob - oa + 1;                  // at most n1 <= kFilterMaxLine
  const bool wrap = !g.window && L >= g.n1;   // a whole periodic line (oa == 0)
  const int vw = vb - va;
  const long long w2 = b.hi[1] - b.lo[1] + 1, rows = w2 * (b.hi[2] - b.lo[2] + 1);
  for (long long r = blockIdx.x; r < 3 * rows; r += gridDim.x) {
    const int comp = (int)(r / rows);
    Real *A = comp == 0 ? A0 : (comp == 1 ? A1 : A2);
    if (!A) continue;  // uniform over the workgroup
    const long long rr = r - comp * rows;
    const int i2 = b.lo[1] + (int)(rr % w2), i3 = b.lo[2] + (int)(rr / w2);
    const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
      const int l = oa + t;
      int d = l - va;
      if (wrap) {
        d %= g.n1;
        d = d < 0 ? d + g.n1 : d;
      }
      line[t] = (d >= 0 && d <= vw) ? A[row + col_of(g, l)] : Real(0);
    }
    __syncthreads();
    for (int p = 0; p <= npass; ++p) {
      const Real a = p < npass ? Real(0.25) : ca, c = p < npass ? Real(0.5) : cb;
      Real v[kFilterPer];
#pragma unroll
      for (int k = 0; k < kFilterPer; ++k) {
        const int t = threadIdx.x + 256 * k;
        if (t < L) {
          const Real lo = t > 0 ? line[t - 1] : (wrap ? line[L - 1] : Real(0));
          const Real hi = t < L - 1 ? line[t + 1] : (wrap ? line[0] : Real(0));
          v[k] = a * lo + c * line[t] + a * hi;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kFilterPer; ++k) {
        const int t = threadIdx.x + 256 * k;
        if (t < L) line[t] = v[k];
      }
      __syncthreads();
    }
    for (int t = threadIdx.x; t < L; t += blockDim.x) A[row + col_of(g, oa + t)] = line[t];
    __syncthreads();
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
__global__ __launch_bounds__(256) void k_new_slab(Geo g, Fields<Real> f, Real *Bx1, Real *Bx2, Real *Bx3, int col,
                                                  Axial<Real> ax) {
  // one wavefront per (x2, x3) row, lanes over the cells the row touches
  const long long r = blockIdx.x * (long long)(blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= (long long)g.n2 * g.n3) return;  // whole wavefront
  const long long row = r * g.n1;
  const long long id = row + col;
  const Real e2b = f.E2[id], e3b = f.E3[id];
  // old window cells j = 1..M-1 reach the leaving cell 0 through C_{j+1}
  if (lane >= 1 && lane < ax.M) {
    const long long k = row + col_of(g, lane);
    f.B2[k] -= ax.c[lane] * e3b;
    f.B3[k] += ax.c[lane] * e2b;
  }
  // new front cell = old window cell n1: d+ f = sum_l C_l (f(n1 + l) - f(n1 - l + 1)),
  // with f zero at old cells >= n1; lane l holds the term of l
  Real s2 = 0, s3 = 0;
  if (lane >= 2 && lane <= ax.M) {
    const long long k = row + col_of(g, g.n1 - lane + 1);
    s2 = ax.c[lane - 1] * f.E2[k];
    s3 = ax.c[lane - 1] * f.E3[k];
  }
  s2 += xor_lane<32>(s2);
  s3 += xor_lane<32>(s3);
  s2 += xor_lane<16>(s2);
  s3 += xor_lane<16>(s3);
  s2 += xor_lane<8>(s2);
  s3 += xor_lane<8>(s3);
  s2 += xor_lane<4>(s2);
  s3 += xor_lane<4>(s3);
  s2 += xor_lane<2>(s2);
  s3 += xor_lane<2>(s3);
  s2 += xor_lane<1>(s2);
  s3 += xor_lane<1>(s3);
  if (lane == 0) {
    f.E1[id] = f.E2[id] = f.E3[id] = Real(0);
    f.B1[id] = Real(0);
    f.B2[id] = s3;   // -d1E3
    f.B3[id] = -s2;  // d1E2
    Bx1[id] = Bx2[id] = Bx3[id] = Real(0);
  }
}

// Window shift after a fused step n (g: geometry before the shift).  The
// fused update took B from n + 1/2 to Bnext = B^{n+1/2} - f dt curl+ E^{n+1}
// (f = 1: B^{n+3/2}; f = 1/2: B^{n+1}) on the old window, where the leaving
// slab (window cell 0, storage column `col`) still holds E^{n+1}; on the
// shifted window that slab is outside and its column is the new front slab.
// The axial stencil is the only part of curl+ that sees the difference:
//   - cells j = 1..M-1 behind the leaving slab: B^{n+1/2} takes the half-step
//     correction of k_new_slab (-ch_j E3, +ch_j E2 on B2, B3, with ch_j =
//     C_{j+1} (dt/2) / dx1), and the f dt curl+ of Bnext loses the leaving
//     slab's term: Bnext gets +(2f - 1) ch_j E3, -(2f - 1) ch_j E2;
//   - the new front column: E^{n+1} = 0, B^{n+1/2} = (0, S3, -S2) with
//     S_c = sum_{l >= 2} ch_{l-1} E_c(old cell n1 - l + 1) as in k_new_slab,
//     and Bnext = (0, (1 - 2f) S3, (2f - 1) S2), its curl+ having only the
//     axial terms reaching back into the window.
// X: B^{n+1/2}, Y: Bnext.  One wavefront per (x2, x3) row.
template <typename Real>
__global__ __launch_bounds__(256) void k_shift_fused(Geo g, Real *E1, Real *E2, Real *E3, Real *X1, Real *X2, Real *X3,
                                                     Real *Y1, Real *Y2, Real *Y3, int col, Axial<Real> ch, Real f2m1) {
  const long long r = blockIdx.x * (long long)(blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= (long long)g.n2 * g.n3) return;  // whole wavefront
  const long long row = r * g.n1;
  const long long id = row + col;
  const Real e2b = E2[id], e3b = E3[id];
  if (lane >= 1 && lane < ch.M) {
    const long long k = row + col_of(g, lane);
    X2[k] -= ch.c[lane] * e3b;
    X3[k] += ch.c[lane] * e2b;
    Y2[k] += f2m1 * (ch.c[lane] * e3b);
    Y3[k] -= f2m1 * (ch.c[lane] * e2b);
  }
  Real s2 = 0, s3 = 0;
  if (lane >= 2 && lane <= ch.M) {
    const long long k = row + col_of(g, g.n1 - lane + 1);
    s2 = ch.c[lane - 1] * E2[k];
    s3 = ch.c[lane - 1] * E3[k];
  }
  s2 += xor_lane<32>(s2);
  s3 += xor_lane<32>(s3);
  s2 += xor_lane<16>(s2);
  s3 += xor_lane<16>(s3);
  s2 += xor_lane<8>(s2);
  s3 += xor_lane<8>(s3);
  s2 += xor_lane<4>(s2);
  s3 += xor_lane<4>(s3);
  s2 += xor_lane<2>(s2);
  s3 += xor_lane<2>(s3);
  s2 += xor_lane<1>(s2);
  s3 += xor_lane<1>(s3);
  if (lane == 0) {
    E1[id] = E2[id] = E3[id] = Real(0);
    X1[id] = Real(0);
    X2[id] = s3;
    X3[id] = -s2;
    Y1[id] = Real(0);
    Y2[id] = -f2m1 * s3;
    Y3[id] = f2m1 * s2;
  }
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
  if (DIM == 3) {
    const unsigned nc = column_blocks(g);
    if (ax.M == 1)
      k_curl_e_col<Real, 1><<<nc, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, h3);
    else if (ax.M == 16)
      k_curl_e_col<Real, 16><<<nc, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, h3);
    else
      k_curl_e_col<Real, 0><<<nc, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, h3);
    return;
  }
  const int rows = rows_per_tile(g);
  const unsigned nb = rows_blocks(g, rows);
  if (ax.M == 1)
    k_curl_e_2d<Real, 1><<<nb, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, rows);
  else if (ax.M == 16)
    k_curl_e_2d<Real, 16><<<nb, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, rows);
  else
    k_curl_e_2d<Real, 0><<<nb, kSeg, 0, st>>>(g, f, Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], ax, h2, rows);
}

template <typename Real, int DIM>
static void curl_b_dispatch(const Geo &g, const Fields<Real> &f, const Axial<Real> &ax, Real e2, Real e3,
                            hipStream_t st) {
  if (DIM == 3) {
    const unsigned nc = column_blocks(g);
    if (ax.M == 1)
      k_curl_b_col<Real, 1><<<nc, kSeg, 0, st>>>(g, f, ax, e2, e3);
    else if (ax.M == 16)
      k_curl_b_col<Real, 16><<<nc, kSeg, 0, st>>>(g, f, ax, e2, e3);
    else
      k_curl_b_col<Real, 0><<<nc, kSeg, 0, st>>>(g, f, ax, e2, e3);
    return;
  }
  const int rows = rows_per_tile(g);
  const unsigned nb = rows_blocks(g, rows);
  if (ax.M == 1)
    k_curl_b_2d<Real, 1><<<nb, kSeg, 0, st>>>(g, f, ax, e2, rows);
  else if (ax.M == 16)
    k_curl_b_2d<Real, 16><<<nb, kSeg, 0, st>>>(g, f, ax, e2, rows);
  else
    k_curl_b_2d<Real, 0><<<nb, kSeg, 0, st>>>(g, f, ax, e2, rows);
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
void launch_clear_j(const Geo &g, const Fields<Real> &f, const JBox *box, int pad, JBox *next, hipStream_t st) {
  k_clear_j<Real><<<1024, 256, 0, st>>>(g, f, box, pad, next);
}

template <typename Real>
void launch_jcorr(const Geo &g, const Real *J1, Real *J1c, const Real *taps, int ng, const JBox *box,
                  hipStream_t st) {
  // a whole x1 line and its taps in LDS when they fit (the box's x1 range
  // is at most n1 after widening)
  const size_t lds = sizeof(Real) * (size_t)(g.n1 + 2 * ng + 1);
  if (lds <= 32768)
    k_jcorr_rows<Real><<<4096, 256, lds, st>>>(g, J1, J1c, taps, ng, box);
  else
    k_jcorr<Real><<<1024, 256, 0, st>>>(g, J1, J1c, taps, ng, box);
}

template <typename Real>
void launch_new_slab(const Geo &g, const Fields<Real> &f, Real *const Bx[3], int col, const Axial<Real> &ax,
                     hipStream_t st) {
  const long long rows = (long long)g.n2 * g.n3;
  k_new_slab<Real><<<(unsigned)((rows + 3) / 4), 256, 0, st>>>(g, f, Bx[0], Bx[1], Bx[2], col, ax);
}

template <typename Real>
void launch_shift_fused(const Geo &g, Real *const E[3], Real *const X[3], Real *const Y[3], int col,
                        const Axial<Real> &ch, Real f2m1, hipStream_t st) {
  const long long rows = (long long)g.n2 * g.n3;
  k_shift_fused<Real><<<(unsigned)((rows + 3) / 4), 256, 0, st>>>(g, E[0], E[1], E[2], X[0], X[1], X[2], Y[0], Y[1],
                                                                    Y[2], col, ch, f2m1);
}

template <typename Real>
void launch_filter_rows(const Geo &g, Real *A0, Real *A1, Real *A2, const JBox *box, int in_pad, int npass, Real ca,
                        Real cb, hipStream_t st) {
  const size_t lds = sizeof(Real) * (size_t)g.n1;  // the widened range is at most one line
  k_filter_rows<Real><<<4096, 256, lds, st>>>(g, A0, A1, A2, box, in_pad, npass, ca, cb);
}

void launch_reset_box(JBox *b, hipStream_t st) { k_reset_box<<<1, 64, 0, st>>>(b); }

#define RELPIC_INST_FIELD(Real)                                                                                   \
  template void launch_curl_e<Real>(int, const Geo &, const Fields<Real> &, Real *const[3], Real *const[3],       \
                                    const Axial<Real> &, Real, Real, hipStream_t);                                \
  template void launch_curl_b<Real>(int, const Geo &, const Fields<Real> &, const Axial<Real> &, Real, Real,      \
                                    hipStream_t);                                                                 \
  template void launch_add_j<Real>(const Geo &, const Fields<Real> &, const Real *, Real, const JBox *, int,     \
                                   JBox *, hipStream_t);                                                          \
  template void launch_clear_j<Real>(const Geo &, const Fields<Real> &, const JBox *, int, JBox *, hipStream_t); \
  template void launch_shift_fused<Real>(const Geo &, Real *const[3], Real *const[3], Real *const[3], int,         \
                                         const Axial<Real> &, Real, hipStream_t);                                 \
  template void launch_jcorr<Real>(const Geo &, const Real *, Real *, const Real *, int, const JBox *,            \
                                   hipStream_t);                                                                  \
  template void launch_filter_rows<Real>(const Geo &, Real *, Real *, Real *, const JBox *, int, int, Real, Real,  \
                                         hipStream_t);                                                            \
  template void launch_new_slab<Real>(const Geo &, const Fields<Real> &, Real *const[3], int, const Axial<Real> &, \
                                      hipStream_t);

RELPIC_INST_FIELD(float)
RELPIC_INST_FIELD(double)

}  // namespace relpic
