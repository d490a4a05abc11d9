// Particle phase of one PIC step (Sec. 1): quadratic-spline gather of E^n,
// B^n at x^n, relativistic Boris push, cell + offset position update and the
// charge-conserving (Esirkepov) current deposit J^{n+1/2}, fused in one pass
// over the particle arrays so each particle's state is read and written once.
//
// Positions are (packed storage cell, offset in [-1/2, 1/2) cell units), so
// FP32 offsets keep full precision at any distance from the origin.
#include "kernels.h"

namespace relpic {

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
  if (o >= Real(0)) {
    qw(o - Real(0.5), w);
    return c;
  }
  qw(o + Real(0.5), w);
  return c - 1;
}

template <typename Real, int DIM>
struct Stagger {
  // node (N) and half (H) stencils per dimension
  int bN[3], bH[3];
  Real wN[3][3], wH[3][3];
};

template <typename Real, int DIM>
__device__ __forceinline__ Real interp(const Geo &g, const Real *f, const Stagger<Real, DIM> &s, const bool h1,
                                       const bool h2, const bool h3) {
  const int b1 = h1 ? s.bH[0] : s.bN[0];
  const int b2 = h2 ? s.bH[1] : s.bN[1];
  const Real *w1 = h1 ? s.wH[0] : s.wN[0];
  const Real *w2 = h2 ? s.wH[1] : s.wN[1];
  int cols[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) cols[a] = col_of(g, b1 - 1 + a);
  Real acc = 0;
  if (DIM == 2) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const long long row = (long long)g.n1 * wrap(b2 - 1 + b, g.n2);
      Real r = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (cols[a] >= 0) r += w1[a] * f[row + cols[a]];
      acc += w2[b] * r;
    }
  } else {
    const int b3 = h3 ? s.bH[2] : s.bN[2];
    const Real *w3 = h3 ? s.wH[2] : s.wN[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int i3 = wrap(b3 - 1 + c, g.n3);
      Real rc = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const long long row = (long long)g.n1 * (wrap(b2 - 1 + b, g.n2) + (long long)g.n2 * i3);
        Real r = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
          if (cols[a] >= 0) r += w1[a] * f[row + cols[a]];
        rc += w2[b] * r;
      }
      acc += w3[c] * rc;
    }
  }
  return acc;
}

// Esirkepov shape arrays on four nodes starting at old cell + base:
// S0 at x^n, DS = S(x^{n+1}) - S(x^n); cum = running sum of DS.
template <typename Real>
__device__ __forceinline__ int esirkepov_1d(Real o0, int sh, Real o1, Real S0[4], Real DS[4], Real cum[4]) {
  Real w0[3], w1[3];
  qw(o0, w0);
  qw(o1, w1);
  const int base = sh < 0 ? -2 : -1;
  Real run = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int k = base + a;        // node relative to the old cell
    const int k1 = k - sh;         // node relative to the new cell
    const Real s0 = (k >= -1 && k <= 1) ? w0[k + 1] : Real(0);
    const Real s1 = (k1 >= -1 && k1 <= 1) ? w1[k1 + 1] : Real(0);
    S0[a] = s0;
    DS[a] = s1 - s0;
    run += DS[a];
    cum[a] = run;
  }
  return base;
}

template <typename Real>
__device__ __forceinline__ void jadd(Real *J, long long idx, Real v) {
  if (v != Real(0)) atomicAdd(J + idx, v);
}

template <typename Real, int DIM>
__global__ __launch_bounds__(256) void k_push_deposit(Geo g, Fields<Real> f, Particles<Real> p, PushParams<Real> q,
                                                      int *err) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const int packed = p.cell[i];
  if (packed < 0) return;
  // decode storage cell -> window cell along x1, rows along x2/x3
  const int s1 = packed % g.n1;
  const int rest = packed / g.n1;
  const int c2 = rest % g.n2;
  const int c3 = DIM == 3 ? rest / g.n2 : 0;
  int c1 = s1 - g.ws_mod;
  if (c1 < 0) c1 += g.n1;
  const int c[3] = {c1, c2, c3};
  const Real o[3] = {p.o1[i], p.o2[i], DIM == 3 ? p.o3[i] : Real(0)};

  // ---- gather E^n, B^n at x^n
  Stagger<Real, DIM> st;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    st.bN[d] = c[d];
    qw(o[d], st.wN[d]);
    st.bH[d] = qw_half(c[d], o[d], st.wH[d]);
  }
  const Real E1 = interp<Real, DIM>(g, f.E1, st, true, false, false);
  const Real E2 = interp<Real, DIM>(g, f.E2, st, false, true, false);
  const Real E3 = interp<Real, DIM>(g, f.E3, st, false, false, true);
  const Real B1 = interp<Real, DIM>(g, f.B1, st, false, true, true);
  const Real B2 = interp<Real, DIM>(g, f.B2, st, true, false, true);
  const Real B3 = interp<Real, DIM>(g, f.B3, st, true, true, false);

  // ---- relativistic Boris push
  const Real a = q.half_qmdt;
  Real um1 = p.u1[i] + a * E1, um2 = p.u2[i] + a * E2, um3 = p.u3[i] + a * E3;
  const Real gm = sqrt(Real(1) + um1 * um1 + um2 * um2 + um3 * um3);
  const Real t1 = a * B1 / gm, t2 = a * B2 / gm, t3 = a * B3 / gm;
  const Real t2s = t1 * t1 + t2 * t2 + t3 * t3;
  const Real f2 = Real(2) / (Real(1) + t2s);
  const Real s1v = f2 * t1, s2v = f2 * t2, s3v = f2 * t3;
  const Real up1 = um1 + (um2 * t3 - um3 * t2);
  const Real up2 = um2 + (um3 * t1 - um1 * t3);
  const Real up3 = um3 + (um1 * t2 - um2 * t1);
  const Real un1 = um1 + (up2 * s3v - up3 * s2v) + a * E1;
  const Real un2 = um2 + (up3 * s1v - up1 * s3v) + a * E2;
  const Real un3 = um3 + (up1 * s2v - up2 * s1v) + a * E3;
  const Real gn = sqrt(Real(1) + un1 * un1 + un2 * un2 + un3 * un3);
  const Real ig = Real(1) / gn;
  if (!(un1 == un1) || !(un2 == un2) || !(un3 == un3)) atomicOr(err, 2);

  // ---- x^{n+1} = x^n + dt u / gamma, in cell units, as cell + offset
  const Real un[3] = {un1, un2, un3};
  int sh[3] = {0, 0, 0};
  Real on[3] = {o[0], o[1], o[2]};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const Real dlt = q.dtdx[d] * un[d] * ig;
    if (!(dlt < Real(1) && dlt > Real(-1))) atomicOr(err, 1);
    Real v = o[d] + dlt;
    int k = 0;
    if (v >= Real(0.5)) k = 1;
    else if (v < Real(-0.5)) k = -1;
    sh[d] = k;
    on[d] = v - Real(k);
  }

  // ---- Esirkepov current J^{n+1/2}
  Real S0[3][4], DS[3][4], cum[3][4];
  int base[3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) base[d] = esirkepov_1d(o[d], sh[d], on[d], S0[d], DS[d], cum[d]);
  int col[4];
#pragma unroll
  for (int aa = 0; aa < 4; ++aa) col[aa] = col_of(g, c1 + base[0] + aa);

  if (DIM == 2) {
    long long row[4];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) row[bb] = (long long)g.n1 * wrap(c2 + base[1] + bb, g.n2);
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const Real wt = q.f1 * (S0[1][bb] + Real(0.5) * DS[1][bb]);
#pragma unroll
      for (int aa = 0; aa < 3; ++aa)
        if (col[aa] >= 0) jadd(f.J1, row[bb] + col[aa], wt * cum[0][aa]);
    }
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) {
      if (col[aa] < 0) continue;
      const Real wt = q.f2 * (S0[0][aa] + Real(0.5) * DS[0][aa]);
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) jadd(f.J2, row[bb] + col[aa], wt * cum[1][bb]);
    }
    const Real jz = q.fv * un3 * ig;
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) {
      if (col[aa] < 0) continue;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const Real w3 = S0[0][aa] * S0[1][bb] + Real(0.5) * DS[0][aa] * S0[1][bb] + Real(0.5) * S0[0][aa] * DS[1][bb] +
                        DS[0][aa] * DS[1][bb] * Real(1.0 / 3.0);
        jadd(f.J3, row[bb] + col[aa], jz * w3);
      }
    }
  } else {
    long long row[4][4];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
        row[cc][bb] =
            (long long)g.n1 * (wrap(c2 + base[1] + bb, g.n2) + (long long)g.n2 * wrap(c3 + base[2] + cc, g.n3));
    const Real third = Real(1.0 / 3.0);
    // J1: transverse weight x running sum of DS1
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const Real wt = q.f1 * (S0[1][bb] * S0[2][cc] + Real(0.5) * DS[1][bb] * S0[2][cc] +
                                Real(0.5) * S0[1][bb] * DS[2][cc] + DS[1][bb] * DS[2][cc] * third);
        if (wt == Real(0)) continue;
#pragma unroll
        for (int aa = 0; aa < 3; ++aa)
          if (col[aa] >= 0) jadd(f.J1, row[cc][bb] + col[aa], wt * cum[0][aa]);
      }
    // J2
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        if (col[aa] < 0) continue;
        const Real wt = q.f2 * (S0[0][aa] * S0[2][cc] + Real(0.5) * DS[0][aa] * S0[2][cc] +
                                Real(0.5) * S0[0][aa] * DS[2][cc] + DS[0][aa] * DS[2][cc] * third);
        if (wt == Real(0)) continue;
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) jadd(f.J2, row[cc][bb] + col[aa], wt * cum[1][bb]);
      }
    // J3
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        if (col[aa] < 0) continue;
        const Real wt = q.f3 * (S0[0][aa] * S0[1][bb] + Real(0.5) * DS[0][aa] * S0[1][bb] +
                                Real(0.5) * S0[0][aa] * DS[1][bb] + DS[0][aa] * DS[1][bb] * third);
        if (wt == Real(0)) continue;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) jadd(f.J3, row[cc][bb] + col[aa], wt * cum[2][cc]);
      }
  }

  // ---- store the new state
  const int n1c = c1 + sh[0];
  int alive = 1;
  if (g.window) {
    const int after = n1c - q.shift;  // window cell after this step's shift
    if (after < 2 || after > g.n1 - 3) alive = 0;
  }
  if (!alive) {
    p.cell[i] = -1;
    return;
  }
  const int ns1 = col_of(g, n1c);
  const int ns2 = wrap(c2 + sh[1], g.n2);
  const int ns3 = DIM == 3 ? wrap(c3 + sh[2], g.n3) : 0;
  p.cell[i] = ns1 + g.n1 * (ns2 + g.n2 * ns3);
  p.o1[i] = on[0];
  p.o2[i] = on[1];
  if (DIM == 3) p.o3[i] = on[2];
  p.u1[i] = un1;
  p.u2[i] = un2;
  p.u3[i] = un3;
}

template <typename Real>
void launch_push_deposit(int ndim, const Geo &g, const Fields<Real> &f, const Particles<Real> &p,
                         const PushParams<Real> &q, int *err, hipStream_t st) {
  if (p.n <= 0) return;
  const unsigned blocks = (unsigned)((p.n + 255) / 256);
  if (ndim == 3)
    k_push_deposit<Real, 3><<<blocks, 256, 0, st>>>(g, f, p, q, err);
  else
    k_push_deposit<Real, 2><<<blocks, 256, 0, st>>>(g, f, p, q, err);
}

template void launch_push_deposit<float>(int, const Geo &, const Fields<float> &, const Particles<float> &,
                                         const PushParams<float> &, int *, hipStream_t);
template void launch_push_deposit<double>(int, const Geo &, const Fields<double> &, const Particles<double> &,
                                          const PushParams<double> &, int *, hipStream_t);

}  // namespace relpic
