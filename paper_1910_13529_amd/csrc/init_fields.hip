// Self-consistent initial fields of charges streaming along x1 (the fields
// Sec. 2.1 gives in terms of the charge density, in the ultra-relativistic
// limit), so that a relativistic beam starts with its own field instead of
// in zero fields (where a static image of opposite charge is left behind and
// the sudden start radiates).
//
// Sec. 2.1: for a particle moving along x1, E2 = i [k]_E2 rho / D and
// B3 = i ([k]_E2/[k]_B1) [w]_t rho / D with D = [w]_t^2 - [k]_E.[k]_B.  For
// a solver whose axial operators satisfy [k]_E1 [k]_B1 = [beta k1]_t^2 (the
// paper's [k]_1 = [k1]_t at beta = 1) D reduces to -[k]_perp^2: in every x1
// slice E_perp is the lattice transverse Poisson field of that slice's charge
// (-lap_perp phi = rho with the Yee transverse operators, E_perp = -grad_perp
// phi), E1 = -(1 - beta^2) d1 phi, and B = beta x E on B's own lattice points
// (B3 at (i1+1/2, i2+1/2) = beta E2 averaged over i1 and i1+1, B2 = -beta E3
// likewise).  The transverse problem is solved by discrete Fourier
// transforms along x2 and x3 (plain sums against a twiddle table, FP64): the
// transforms run once, at set-up, not in the PIC step.  The x2/x3-uniform
// part of each slice's charge (zero for a beam neutralized by a co-moving,
// transversely uniform charge) has no transverse field and is left out.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "engine.h"

using namespace relpic;
using namespace relpic_host;

namespace {

constexpr int kInitBlock = 256;

// out(i1, k, ..) = sum_j in(i1, j, ..) exp(sign 2 pi i j k / n) along x2
// (axis 1) or x3 (axis 2); tw[m] = (cos, sin)(2 pi m / n)
__global__ __launch_bounds__(kInitBlock) void k_dft_axis(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                        int n1, int n2, int n3, int axis, double sign,
                                                        const double2 *__restrict__ tw) {
  const long long N = (long long)n1 * n2 * n3;
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= N) return;
  const int i1 = (int)(idx % n1);
  const long long q = idx / n1;
  const int i2 = (int)(q % n2);
  const int i3 = (int)(q / n2);
  const int n = axis == 1 ? n2 : n3;
  const int k = axis == 1 ? i2 : i3;
  const long long stride = axis == 1 ? (long long)n1 : (long long)n1 * n2;
  const long long base = axis == 1 ? i1 + (long long)n1 * n2 * i3 : i1 + (long long)n1 * i2;
  double re = 0.0, im = 0.0;
  int m = 0;  // (j k) mod n
  for (int j = 0; j < n; ++j) {
    const double2 v = in[base + j * stride];
    const double2 w = tw[m];
    const double ws = sign * w.y;
    re += v.x * w.x - v.y * ws;
    im += v.x * ws + v.y * w.x;
    m += k;
    if (m >= n) m -= n;
  }
  out[idx] = make_double2(re, im);
}

// rho (storage layout) -> complex
__global__ __launch_bounds__(kInitBlock) void k_to_complex(const double *__restrict__ rho, double2 *__restrict__ out,
                                                          long long N) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < N) out[i] = make_double2(rho[i], 0.0);
}

// phi_hat = rho_hat / (s2^2 + s3^2), s_d = 2 sin(pi k_d / n_d) / dx_d; the
// transversely uniform mode (k2 = k3 = 0) is dropped
__global__ __launch_bounds__(kInitBlock) void k_poisson(double2 *__restrict__ a, int n1, int n2, int n3, double dx2,
                                                       double dx3, int ndim) {
  const long long N = (long long)n1 * n2 * n3;
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= N) return;
  const long long q = idx / n1;
  const int k2 = (int)(q % n2);
  const int k3 = (int)(q / n2);
  const double s2 = 2.0 * sin(M_PI * k2 / n2) / dx2;
  const double s3 = ndim == 3 ? 2.0 * sin(M_PI * k3 / n3) / dx3 : 0.0;
  const double den = s2 * s2 + s3 * s3;
  double2 v = a[idx];
  if (den > 0.0) {
    v.x /= den;
    v.y /= den;
  } else {
    v = make_double2(0.0, 0.0);
  }
  a[idx] = v;
}

// fields from phi (real part of the inverse transform, times `scale`) on
// their staggered points; storage layout with the ring-buffer x1 columns
template <typename Real>
__global__ __launch_bounds__(kInitBlock) void k_beam_fields(Geo g, const double2 *__restrict__ phi, double scale,
                                                           double beta, double idx1, double idx2, double idx3,
                                                           int ndim, Fields<Real> f) {
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= g.N) return;
  const int s1 = (int)(idx % g.n1);
  const long long q = idx / g.n1;
  const int i2 = (int)(q % g.n2);
  const int i3 = (int)(q / g.n2);
  // window cell of this column and its +x1 neighbour (zero beyond the window)
  int l = s1 - g.ws_mod;
  if (l < 0) l += g.n1;
  const bool has_next = !g.window || l + 1 < g.n1;
  const int sn = s1 + 1 == g.n1 ? 0 : s1 + 1;
  auto P = [&](int c1, int c2, int c3) -> double {
    return phi[c1 + (long long)g.n1 * (c2 + (long long)g.n2 * c3)].x * scale;
  };
  const int p2 = i2 + 1 == g.n2 ? 0 : i2 + 1;
  const int p3 = ndim == 3 ? (i3 + 1 == g.n3 ? 0 : i3 + 1) : 0;
  const double ph = P(s1, i2, i3);
  const double phn = has_next ? P(sn, i2, i3) : 0.0;
  const double e2 = -(P(s1, p2, i3) - ph) * idx2;
  const double e2n = has_next ? -(P(sn, p2, i3) - phn) * idx2 : 0.0;
  double e3 = 0.0, e3n = 0.0;
  if (ndim == 3) {
    e3 = -(P(s1, i2, p3) - ph) * idx3;
    e3n = has_next ? -(P(sn, i2, p3) - phn) * idx3 : 0.0;
  }
  const double e1 = -(1.0 - beta * beta) * (phn - ph) * idx1;
  f.E1[idx] = (Real)e1;
  f.E2[idx] = (Real)e2;
  f.E3[idx] = (Real)e3;
  f.B1[idx] = Real(0);
  f.B2[idx] = (Real)(-beta * 0.5 * (e3 + e3n));
  f.B3[idx] = (Real)(beta * 0.5 * (e2 + e2n));
}

unsigned blocks_for(long long n) { return (unsigned)((n + kInitBlock - 1) / kInitBlock); }

template <typename Real>
relpic_status init_fields(relpic_sim *s, double beta) {
  const Geo g = make_geo(s);
  const long long N = s->N;
  const int n2 = s->n[1], n3 = s->n[2];
  const double dV = cell_volume(s);
  HIP_OK(hipMemsetAsync(s->rho, 0, sizeof(double) * N, s->st));
  for (auto &sp : s->sp) launch_diag_rho<Real>(s->ndim, g, parts<Real>(sp), sp.Q / dV, s->rho, s->st);
  double2 *a = (double2 *)dev_alloc(s, sizeof(double2) * N);
  double2 *b = (double2 *)dev_alloc(s, sizeof(double2) * N);
  double2 *tw = (double2 *)dev_alloc(s, sizeof(double2) * (size_t)(n2 + n3));
  if (!a || !b || !tw) return fail(RELPIC_ENOMEM, "init_beam_fields: allocation failed");
  std::vector<double2> htw((size_t)(n2 + n3));
  for (int m = 0; m < n2; ++m) htw[m] = make_double2(std::cos(2.0 * M_PI * m / n2), std::sin(2.0 * M_PI * m / n2));
  for (int m = 0; m < n3; ++m)
    htw[n2 + m] = make_double2(std::cos(2.0 * M_PI * m / n3), std::sin(2.0 * M_PI * m / n3));
  HIP_OK(hipMemcpyAsync(tw, htw.data(), sizeof(double2) * htw.size(), hipMemcpyHostToDevice, s->st));
  const unsigned nb = blocks_for(N);
  k_to_complex<<<nb, kInitBlock, 0, s->st>>>(s->rho, a, N);
  k_dft_axis<<<nb, kInitBlock, 0, s->st>>>(a, b, s->n[0], n2, n3, 1, -1.0, tw);
  double2 *cur = b, *oth = a;
  if (s->ndim == 3) {
    k_dft_axis<<<nb, kInitBlock, 0, s->st>>>(b, a, s->n[0], n2, n3, 2, -1.0, tw + n2);
    cur = a;
    oth = b;
  }
  k_poisson<<<nb, kInitBlock, 0, s->st>>>(cur, s->n[0], n2, n3, s->dx[1], s->ndim == 3 ? s->dx[2] : 1.0, s->ndim);
  if (s->ndim == 3) {
    k_dft_axis<<<nb, kInitBlock, 0, s->st>>>(cur, oth, s->n[0], n2, n3, 2, 1.0, tw + n2);
    std::swap(cur, oth);
  }
  k_dft_axis<<<nb, kInitBlock, 0, s->st>>>(cur, oth, s->n[0], n2, n3, 1, 1.0, tw);
  const double scale = 1.0 / ((double)n2 * (s->ndim == 3 ? n3 : 1));
  k_beam_fields<Real><<<nb, kInitBlock, 0, s->st>>>(g, oth, scale, beta, 1.0 / s->dx[0], 1.0 / s->dx[1],
                                                   s->ndim == 3 ? 1.0 / s->dx[2] : 0.0, s->ndim, fields<Real>(s));
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s->st));
  dev_release(s, a);
  dev_release(s, b);
  dev_release(s, tw);
  return RELPIC_OK;
}

}  // namespace

extern "C" {

relpic_status relpic_init_beam_fields(relpic_sim *s, double beta) {
  return guarded("init_beam_fields", [&]() -> relpic_status {
    if (!s) return fail(RELPIC_EINVAL, "null simulation handle");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(RELPIC_EINVAL, "init_beam_fields: need 0 < beta <= 1");
    if (s->step != 0) return fail(RELPIC_ESTATE, "init_beam_fields: only before the first step");
    return s->prec == RELPIC_FP32 ? init_fields<float>(s, beta) : init_fields<double>(s, beta);
  });
}

}  // extern "C"
