// Fused leapfrog field advance for 3D grids whose x1 lines fit one workgroup
// (Eq. 1 with the operators of Eq. 14 and, along x1, the customized 2M-point
// operator of App. C).  One launch takes E from step n to n + 1 and B from
// n + 1/2 to the next B time:
//   E^{n+1} = E^n + dt d- x B^{n+1/2} - dt J^{n+1/2}  (J inside the deposit box, J1 corrected)
//   Bnext   = B^{n+1/2} - f dt d+ x E^{n+1}            (f = 1: B^{n+3/2}; f = 1/2: B^{n+1})
// Every field word is read once and written once: 12 words per cell against
// the 18 of the two separate updates.  E^{n+1} goes to a second E buffer, as
// neighbouring workgroups still read E^n; B goes to the buffer that held
// B^{n-1/2}.  The arithmetic per cell is that of k_curl_b_col, k_add_j and
// k_curl_e_col, in the same order.
//
// A workgroup owns R consecutive x2 rows of whole x1 lines (thread t holds
// window cell t of every row) and marches through `planes` x3 planes.  B at
// (row j, plane k) needs E^{n+1} at row j + 1 and at plane k + 1, so the B
// update runs one plane behind the E update, and the workgroup also computes
// E^{n+1} on the first row of the next row block (E1, E3) and on the first
// plane of the next column, without storing them.  Each x1 line is staged in
// LDS with a halo of H cells per side (periodic copies, or zeros outside a
// moving window).
#include "field_tiles.h"

namespace relpic {

namespace {

// planes per workgroup: long enough columns that about two workgroups per CU
// cover the grid in one round (the recomputed plane is 1/planes of the work),
// at least 8
constexpr int kLeapWorkgroups = 512;

inline int leap_planes(const Geo &g, int R) {
  const long long nrb = g.n2 / R;
  long long p = (nrb * g.n3 + kLeapWorkgroups - 1) / kLeapWorkgroups;
  if (p < 8) p = 8;
  if (p > g.n3) p = g.n3;
  return (int)p;
}

// x2 rows per workgroup: more rows share the recomputed neighbour row, fewer
// keep the per-plane operands in registers at 4 waves per SIMD (FP32: 121
// VGPRs at two rows, 204 at four; FP64: 186 at two rows, so one)
template <typename Real>
struct LeapRows {
  static constexpr int R = 2;
};
template <>
struct LeapRows<double> {
  static constexpr int R = 1;
};

template <typename Real, int R>
struct LeapPlane {
  Real b1[R + 2], b3[R + 2];  // rows -1 .. R
  Real b2[R + 1];             // rows 0 .. R
  Real e1[R + 1], e3[R + 1];  // rows 0 .. R
  Real e2[R];                 // rows 0 .. R - 1
};

template <typename Real, int MM, int R>
__global__ __launch_bounds__(512) void k_leap(Geo g, const Real *__restrict__ Ei1, const Real *__restrict__ Ei2,
                                               const Real *__restrict__ Ei3, Real *__restrict__ Eo1,
                                               Real *__restrict__ Eo2, Real *__restrict__ Eo3,
                                               const Real *__restrict__ B1, const Real *__restrict__ B2,
                                               const Real *__restrict__ B3, Real *__restrict__ Bo1,
                                               Real *__restrict__ Bo2, Real *__restrict__ Bo3, const Real *J1s,
                                               const Real *J2, const Real *J3, const JBox *jbox, int pad, Real dt,
                                               Axial<Real> axE, Real e2c, Real e3c, Axial<Real> axB, Real h2,
                                               Real h3, int planes) {
  extern __shared__ __align__(16) unsigned char leap_lds[];
  constexpr int H = MM > 0 ? MM : kMaxM;  // staged halo per side
  const int M = MM > 0 ? MM : axE.M;
  const int pitch = g.n1 + 2 * H;
  Real *sB2 = reinterpret_cast<Real *>(leap_lds);  // R + 1 rows
  Real *sB3 = sB2 + (R + 1) * pitch;                // R rows
  Real *sE2 = sB3 + R * pitch;                      // R rows
  Real *sE3 = sE2 + R * pitch;                      // R rows

  // tile: rows r0 .. r0 + R - 1 of planes z0 .. z1 - 1; each XCD takes a
  // contiguous band of tiles, so row blocks that share a row run side by side
  const int nrb = g.n2 / R;
  const int nz = (g.n3 + planes - 1) / planes;
  const long long nb = (long long)nrb * nz;
  const long long per = (nb + kNumXcd - 1) / kNumXcd;
  const long long lin = (blockIdx.x % kNumXcd) * per + blockIdx.x / kNumXcd;
  if (lin >= nb) return;  // whole workgroup, before any barrier
  const int r0 = (int)(lin % nrb) * R;
  const int z0 = (int)(lin / nrb) * planes;
  const int z1 = min(z0 + planes, g.n3);

  const int t = threadIdx.x;
  const bool own = t < g.n1;
  const int s1 = own ? col_near(g, t) : 0;
  const int c = t + H;  // LDS index of window cell t
  const long long plane = (long long)g.n1 * g.n2;
  long long roff[R + 2];  // storage offsets of rows r0 - 1 .. r0 + R within a plane (own column)
#pragma unroll
  for (int j = 0; j < R + 2; ++j) roff[j] = (long long)g.n1 * wrap_near(r0 - 1 + j, g.n2) + s1;

  // deposit box: rows, planes and (widened) window cells where J is added
  const JBox jb = *jbox;
  int lo1 = 0, hi1 = -1;
  const bool anyj = box_x1(g, jb, pad, lo1, hi1);
  const bool jcol = anyj && t >= lo1 && t <= hi1;

  if (g.window)
    for (int q = t; q < (4 * R + 1) * 2 * H; q += blockDim.x) {
      const int row = q / (2 * H), h = q - row * 2 * H;
      sB2[row * pitch + (h < H ? h : g.n1 + h)] = Real(0);
    }
  auto stage = [&](Real *row, Real v) {
    if (own) {
      row[c] = v;
      if (!g.window) {
        if (t < H) row[c + g.n1] = v;
        if (t >= g.n1 - H) row[c - g.n1] = v;
      }
    }
  };
  auto fetch = [&](LeapPlane<Real, R> &P, int k) {
    if (!own) return;
    const long long po = plane * wrap_near(k, g.n3);
#pragma unroll
    for (int j = 0; j < R + 2; ++j) {
      P.b1[j] = B1[po + roff[j]];
      P.b3[j] = B3[po + roff[j]];
    }
#pragma unroll
    for (int j = 0; j <= R; ++j) {
      P.b2[j] = B2[po + roff[j + 1]];
      P.e1[j] = Ei1[po + roff[j + 1]];
      P.e3[j] = Ei3[po + roff[j + 1]];
    }
#pragma unroll
    for (int j = 0; j < R; ++j) P.e2[j] = Ei2[po + roff[j + 1]];
  };

  LeapPlane<Real, R> cur, nxt;
#pragma unroll
  for (int j = 0; j < R + 2; ++j) cur.b1[j] = cur.b3[j] = Real(0);
#pragma unroll
  for (int j = 0; j <= R; ++j) cur.b2[j] = cur.e1[j] = cur.e3[j] = Real(0);
#pragma unroll
  for (int j = 0; j < R; ++j) cur.e2[j] = Real(0);
  nxt = cur;
  // B1, B2 of plane z0 - 1 (x3 differences of E^{n+1} at z0)
  Real b1p[R], b2p[R + 1];
#pragma unroll
  for (int j = 0; j < R; ++j) b1p[j] = Real(0);
#pragma unroll
  for (int j = 0; j <= R; ++j) b2p[j] = Real(0);
  if (own) {
    const long long po = plane * wrap_near(z0 - 1, g.n3);
#pragma unroll
    for (int j = 0; j < R; ++j) b1p[j] = B1[po + roff[j + 1]];
#pragma unroll
    for (int j = 0; j <= R; ++j) b2p[j] = B2[po + roff[j + 1]];
  }
  fetch(cur, z0);
  // E^{n+1} and B^{n+1/2} (own rows) of the previous plane
  Real pE1[R + 1], pE2[R], pE3[R + 1], ob1[R], ob2[R], ob3[R];
#pragma unroll
  for (int j = 0; j <= R; ++j) pE1[j] = pE3[j] = Real(0);
#pragma unroll
  for (int j = 0; j < R; ++j) pE2[j] = ob1[j] = ob2[j] = ob3[j] = Real(0);

  for (int k = z0; k <= z1; ++k) {
    const int kw = wrap_near(k, g.n3);
    // Wave priorities along a plane: staging 2 (the barrier is reached
    // sooner; 0.394 -> 0.381 ms), the next plane's loads 3, the E update 0,
    // the B update 1.
    __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int j = 0; j <= R; ++j) stage(sB2 + j * pitch, cur.b2[j]);
#pragma unroll
    for (int j = 0; j < R; ++j) stage(sB3 + j * pitch, cur.b3[j + 1]);
    if (k > z0) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        stage(sE2 + j * pitch, pE2[j]);
        stage(sE3 + j * pitch, pE3[j]);
      }
    }
    __syncthreads();
    // the next plane's loads go out at raised wave priority, so waves leaving
    // the barrier issue them before the LDS stencil work of the others
    // (0.409 -> 0.394 ms on the 3D beam)
    __builtin_amdgcn_s_setprio(3);
    if (k < z1) fetch(nxt, k + 1);
    __builtin_amdgcn_s_setprio(0);
    const bool jplane = anyj && kw >= jb.lo[2] && kw <= jb.hi[2];
    // E^{n+1} of plane k, rows 0 .. R (row R: E1, E3 only)
    Real nE1[R + 1], nE2[R], nE3[R + 1];
#pragma unroll
    for (int j = 0; j <= R; ++j) nE1[j] = nE3[j] = Real(0);
#pragma unroll
    for (int j = 0; j < R; ++j) nE2[j] = Real(0);
    if (own) {
#pragma unroll
      for (int j = 0; j <= R; ++j) {
        const Real *rB2 = sB2 + j * pitch;
        Real d1B2 = 0;
        auto term2 = [&](int l) { d1B2 += axE.c[l - 1] * (rB2[c + l - 1] - rB2[c - l]); };
        if (MM > 0) {
#pragma unroll
          for (int l = 1; l <= MM; ++l) term2(l);
        } else {
          for (int l = 1; l <= M; ++l) term2(l);
        }
        const Real d2B3 = e2c * (cur.b3[j + 1] - cur.b3[j]);
        const Real d3B2 = e3c * (cur.b2[j] - b2p[j]);
        const Real d2B1 = e2c * (cur.b1[j + 1] - cur.b1[j]);
        Real x1 = cur.e1[j] + (d2B3 - d3B2);
        Real x3 = cur.e3[j] + (d1B2 - d2B1);
        Real x2 = 0;
        if (j < R) {
          const Real *rB3 = sB3 + j * pitch;
          Real d1B3 = 0;
          auto term3 = [&](int l) { d1B3 += axE.c[l - 1] * (rB3[c + l - 1] - rB3[c - l]); };
          if (MM > 0) {
#pragma unroll
            for (int l = 1; l <= MM; ++l) term3(l);
          } else {
            for (int l = 1; l <= M; ++l) term3(l);
          }
          const Real d3B1 = e3c * (cur.b1[j + 1] - b1p[j]);
          x2 = cur.e2[j] + (d3B1 - d1B3);
        }
        if (jplane && jcol) {
          const int rw = wrap_near(r0 + j, g.n2);
          if (rw >= jb.lo[1] && rw <= jb.hi[1]) {
            const long long id = plane * kw + roff[j + 1];
            x1 -= dt * J1s[id];
            x3 -= dt * J3[id];
            if (j < R) x2 -= dt * J2[id];
          }
        }
        nE1[j] = x1;
        nE3[j] = x3;
        if (j < R) nE2[j] = x2;
      }
    }
    // the B update (and the E stores) at priority 1: waves further along
    // the plane go first, so the end-of-plane barrier comes sooner
    // (0.382 -> 0.362 ms)
    __builtin_amdgcn_s_setprio(1);
    // B of plane k - 1 from E^{n+1} of planes k - 1 (staged) and k
    if (k > z0 && own) {
      const long long po = plane * (k - 1);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const Real *rE2 = sE2 + j * pitch, *rE3 = sE3 + j * pitch;
        Real d1E2 = 0, d1E3 = 0;
        auto term = [&](int l) {
          d1E2 += axB.c[l - 1] * (rE2[c + l] - rE2[c - l + 1]);
          d1E3 += axB.c[l - 1] * (rE3[c + l] - rE3[c - l + 1]);
        };
        if (MM > 0) {
#pragma unroll
          for (int l = 1; l <= MM; ++l) term(l);
        } else {
          for (int l = 1; l <= M; ++l) term(l);
        }
        const Real e1 = pE1[j], e2 = pE2[j], e3 = pE3[j];
        const Real d2E3 = h2 * (pE3[j + 1] - e3);
        const Real d2E1 = h2 * (pE1[j + 1] - e1);
        const Real d3E2 = h3 * (nE2[j] - e2);
        const Real d3E1 = h3 * (nE1[j] - e1);
        const long long id = po + roff[j + 1];
        Bo1[id] = ob1[j] - (d2E3 - d3E2);
        Bo2[id] = ob2[j] - (d3E1 - d1E3);
        Bo3[id] = ob3[j] - (d1E2 - d2E1);
      }
    }
    if (k < z1 && own) {
      const long long po = plane * k;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const long long id = po + roff[j + 1];
        Eo1[id] = nE1[j];
        Eo2[id] = nE2[j];
        Eo3[id] = nE3[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j <= R; ++j) {
      pE1[j] = nE1[j];
      pE3[j] = nE3[j];
      b2p[j] = cur.b2[j];
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      pE2[j] = nE2[j];
      b1p[j] = cur.b1[j + 1];
      ob1[j] = cur.b1[j + 1];
      ob2[j] = cur.b2[j];
      ob3[j] = cur.b3[j + 1];
    }
    cur = nxt;
  }
}

template <typename Real, int R>
void leap_dispatch(const Geo &g, Real *const Ein[3], Real *const Eout[3], Real *const Bin[3], Real *const Bout[3],
                   const Real *J1s, const Real *J2, const Real *J3, const JBox *box, int pad, Real dt,
                   const Axial<Real> &axE, Real e2c, Real e3c, const Axial<Real> &axB, Real h2, Real h3,
                   hipStream_t st) {
  const int H = (axE.M == 1 || axE.M == 16) ? axE.M : kMaxM;
  const size_t lds = sizeof(Real) * (size_t)(4 * R + 1) * (size_t)(g.n1 + 2 * H);
  const unsigned threads = (unsigned)((g.n1 + 63) / 64 * 64);
  const int planes = leap_planes(g, R);
  const long long nb = (long long)(g.n2 / R) * ((g.n3 + planes - 1) / planes);
  const unsigned blocks = (unsigned)((nb + kNumXcd - 1) / kNumXcd * kNumXcd);
#define RELPIC_LEAP_ARGS                                                                                        \
  g, Ein[0], Ein[1], Ein[2], Eout[0], Eout[1], Eout[2], Bin[0], Bin[1], Bin[2], Bout[0], Bout[1], Bout[2], J1s, J2, \
      J3, box, pad, dt, axE, e2c, e3c, axB, h2, h3, planes
  if (axE.M == 1)
    k_leap<Real, 1, R><<<blocks, threads, lds, st>>>(RELPIC_LEAP_ARGS);
  else if (axE.M == 16)
    k_leap<Real, 16, R><<<blocks, threads, lds, st>>>(RELPIC_LEAP_ARGS);
  else
    k_leap<Real, 0, R><<<blocks, threads, lds, st>>>(RELPIC_LEAP_ARGS);
#undef RELPIC_LEAP_ARGS
}

}  // namespace

template <typename Real>
bool leap_supported(const Geo &g, int M) {
  constexpr int R = LeapRows<Real>::R;
  const int H = (M == 1 || M == 16) ? M : kMaxM;
  const size_t lds = sizeof(Real) * (size_t)(4 * R + 1) * (size_t)(g.n1 + 2 * H);
  return g.n3 > 1 && g.n1 <= 512 && g.n1 >= 2 * H && g.n2 % R == 0 && lds <= 65536;
}

template <typename Real>
void launch_leap(const Geo &g, Real *const Ein[3], Real *const Eout[3], Real *const Bin[3], Real *const Bout[3],
                 const Real *J1s, const Real *J2, const Real *J3, const JBox *box, int pad, Real dt,
                 const Axial<Real> &axE, Real e2c, Real e3c, const Axial<Real> &axB, Real h2, Real h3,
                 hipStream_t st) {
  leap_dispatch<Real, LeapRows<Real>::R>(g, Ein, Eout, Bin, Bout, J1s, J2, J3, box, pad, dt, axE, e2c, e3c, axB, h2,
                                         h3, st);
}

#define RELPIC_INST_LEAP(Real)                                                                                  \
  template bool leap_supported<Real>(const Geo &, int);                                                         \
  template void launch_leap<Real>(const Geo &, Real *const[3], Real *const[3], Real *const[3], Real *const[3],  \
                                  const Real *, const Real *, const Real *, const JBox *, int, Real,             \
                                  const Axial<Real> &, Real, Real, const Axial<Real> &, Real, Real, hipStream_t);

RELPIC_INST_LEAP(float)
RELPIC_INST_LEAP(double)

}  // namespace relpic
