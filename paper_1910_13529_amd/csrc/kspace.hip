// The paper's k-space field of a charge streaming along x1 (Sec. 2, Eq. 13;
// general beta through Eqs. 8-9), evaluated by FP64 quadrature on the GPU.
//
// On axis, at the E1 point i1' cells from the particle (E1 at i1' + 1/2), in
// normalized variables khat = k1 dx1 / 2, theta = k2 dx2 / 2, r = dx2/dx1,
// kappa = dx1/dt:
//   E1 dx1 / q = -1/(2 pi^2 r) sum_nu int_{-pi/2}^{pi/2} dkhat
//                Re[ (i / sigma1(khat)) Shat(khat + nu pi) I_nu(khat) e^{i khat (2 i1' + 1)} ]
//   sigma1 = [k]_1 dx1 / 2 = sum_l C_l sin((2l - 1) khat)   (Yee: sin khat)
//   Shat(k) = (sin k / k)^(p + 1)                            (B-spline of order p)
//   A = r^2 (tau^2 - sigma1^2),  tau = kappa sin(beta (khat + nu pi) / kappa)
//   I_nu = int_{-pi/2}^{pi/2} dtheta T(theta)^q A / (A - sin^2 theta)
// with the Yee transverse operator and T = 1 - sin^2(theta)/2 the transverse
// density factor of a quadratic deposit (q = 0: the paper's linear shape,
// whose aliases sum to 1).  App. D gives the theta integral in closed form:
//   q = 0: I = pi sqrt(A / (A - 1))               (A < 0 or A > 1)
//          I = -i s pi sqrt(A / (1 - A))          (0 < A < 1, causal pole)
// with s = sign(sin(beta k1' dt)), and writing T = h + (A - sin^2)/2,
// h = 1 - A/2, polynomial division gives
//   q = 1: h I0 + pi A / 2
//   q = 2: h^2 I0 + h pi A + (A/4)(pi A - pi/2).
// The self-force (Eqs. 19, 25) weights the same integrand by the gather's
// unaliased shape Shat_g(khat) instead of the staggering phase.
//
// Off axis (E1 at transverse node i2) the theta integral carries
// cos(2 i2 theta); by residues, with phi = 2 theta and a = 2A - 1,
//   int_{-pi}^{pi} cos(n phi) / (a + cos phi) dphi = 2 pi z^|n| / w,  z = w - a,
// w = sign(a) sqrt(a^2 - 1) for |a| > 1 and w = i s sqrt(1 - a^2) on the
// pole (the causal root), and T = (3 + cos phi)/4 is divided out by
// polynomial division (k2n).  In 3D (Eq. 9 with both transverse
// integrals),
//   E1 dx1^2 / q = -1/(2 pi^3 r2 r3) sum_nu int dkhat
//                  Re[(i / sigmaB) Shat I3 e^{i khat (2 i1' + 1)}],
//   I3 = 2 r3^2 X int_0^{pi/2} dtheta2 T2 cos(2 i2 theta2) J(r3^2 (X - sin^2 theta2 / r2^2)),
// X = tau^2 - sigmaE sigmaB and J(A) = k2n(A) / A the x3 integral without
// its factor A; the theta2 integral is tanh-sinh on panels split where its
// argument crosses 0 and 1 (closed form), inside every k1 node.
//
// The host splits [-pi/2, pi/2] of each zone nu at every point where the
// integrand is singular or changes form (A = 0, A = 1, sin(beta k1' dt) = 0,
// khat = 0); the device integrates each panel with tanh-sinh quadrature,
// whose nodes crowd double-exponentially at the panel ends, so the
// integrable 1/sqrt(1 - A) end singularities converge without special care.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"

using namespace relpic;
using namespace relpic_host;

namespace {

constexpr int kKsMaxM = 32;
constexpr double kPi = 3.14159265358979323846;
constexpr double kTsStep = 1.0 / 64.0;  // tanh-sinh step
constexpr int kTsHalf = 224;            // nodes k = -kTsHalf .. kTsHalf (t up to 3.5)

struct KsParams {
  int M;
  double C[kKsMaxM];   // operator on E, [k]_E1
  double CB[kKsMaxM];  // operator on B, [k]_B1 (zero-padded to M)
  double kappa, r, beta;
  int order, tpow, gather_order;
  double r3;  // dx3 / dx1 (3D)
};

struct Panel {
  double a, b;
  int nu;
  int pad_;
};

__host__ __device__ inline double sigma1(const KsParams &p, double kh) {
  double v = 0.0;
  for (int l = 1; l <= p.M; ++l) v += p.C[l - 1] * sin((2 * l - 1) * kh);
  return v;
}

__host__ __device__ inline double sigma1b(const KsParams &p, double kh) {
  double v = 0.0;
  for (int l = 1; l <= p.M; ++l) v += p.CB[l - 1] * sin((2 * l - 1) * kh);
  return v;
}

__host__ __device__ inline double a_of(const KsParams &p, double kh, int nu) {
  const double tau = p.kappa * sin(p.beta * (kh + nu * kPi) / p.kappa);
  return p.r * p.r * (tau * tau - sigma1(p, kh) * sigma1b(p, kh));
}

__device__ inline double shat(double k, int order) {
  const double s = k == 0.0 ? 1.0 : sin(k) / k;
  double v = s;
  for (int i = 0; i < order; ++i) v *= s;
  return v;
}

// k2 integral: returns (re, im)
__device__ inline void k2_integral(double A, double s, int tpow, double &re, double &im) {
  re = im = 0.0;
  if (A == 0.0) return;
  double br = 0.0, bi = 0.0;
  if (A < 0.0 || A > 1.0)
    br = kPi * sqrt(A / (A - 1.0));
  else
    bi = -s * kPi * sqrt(A / (1.0 - A));
  if (tpow == 0) {
    re = br;
    im = bi;
    return;
  }
  const double h = 1.0 - 0.5 * A;
  if (tpow == 1) {
    re = h * br + 0.5 * kPi * A;
    im = h * bi;
    return;
  }
  re = h * h * br + h * kPi * A + 0.25 * A * (kPi * A - 0.5 * kPi);
  im = h * h * bi;
}

struct Cplx {
  double re, im;
};
__device__ inline Cplx cmul(Cplx a, Cplx b) { return Cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cplx cdiv(Cplx a, Cplx b) {
  const double d = b.re * b.re + b.im * b.im;
  return Cplx{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// Off-axis theta integral divided by A:
//   J_n(A) = int_{-pi/2}^{pi/2} dtheta T^tpow cos(2 n theta) / (A + i0 s - sin^2 theta)
// (so that the 2D integrand's Ihat_n = A J_n); zero at the integrable
// branch points A = 0, 1 themselves
__device__ inline Cplx k2n_over_a(double A, double s, int tpow, int n) {
  n = n < 0 ? -n : n;
  const double a = 2.0 * A - 1.0;
  Cplx w;
  if (fabs(a) > 1.0)
    w = Cplx{copysign(sqrt(a * a - 1.0), a), 0.0};
  else
    w = Cplx{0.0, s * sqrt(1.0 - a * a)};
  if (w.re == 0.0 && w.im == 0.0) return Cplx{0.0, 0.0};
  const Cplx z{w.re - a, w.im};
  Cplx zn{1.0, 0.0};
  for (int k = 0; k < n; ++k) zn = cmul(zn, z);
  Cplx In = cdiv(zn, w);  // int_{-pi}^{pi} cos(n phi) / (a + cos phi) dphi = 2 pi z^n / w
  In.re *= 2.0 * kPi;
  In.im *= 2.0 * kPi;
  const double d0 = n == 0 ? 2.0 * kPi : 0.0, d1 = n == 1 ? kPi : 0.0;
  // theta -> phi = 2 theta turns dtheta / (A - sin^2) into dphi / (a + cos phi)
  Cplx J;
  if (tpow == 0) {
    J = In;
  } else if (tpow == 1) {
    J = Cplx{0.25 * (d0 + (3.0 - a) * In.re), 0.25 * (3.0 - a) * In.im};
  } else {
    const double c = (3.0 - a) * (3.0 - a) / 16.0;
    J = Cplx{(a * d0 + d1 + 2.0 * (3.0 - a) * d0) / 16.0 + c * In.re, c * In.im};
  }
  return J;
}

// tanh-sinh rule of the inner (theta2) integral: step 1/32, t up to 3
constexpr double kTsStepIn = 1.0 / 32.0;
constexpr int kTsHalfIn = 96;

// I3 of zone nu at khat (3D transverse integral, x3 closed form, x2 tanh-sinh)
__device__ inline Cplx i3_integral(const KsParams &p, double X, double s, int i2, int i3) {
  if (X == 0.0) return Cplx{0.0, 0.0};
  const double r2 = p.r, r3 = p.r3;
  // panels of [0, pi/2]: split where r3^2 (X - sin^2 / r2^2) = 0 or 1
  double bp[4];
  int nb = 0;
  bp[nb++] = 0.0;
  const double v0 = r2 * r2 * X, v1 = r2 * r2 * (X - 1.0 / (r3 * r3));
  // v1 < v0, so the A3 = 1 point comes first
  if (v1 > 0.0 && v1 < 1.0) bp[nb++] = asin(sqrt(v1));
  if (v0 > 0.0 && v0 < 1.0) bp[nb++] = asin(sqrt(v0));
  bp[nb++] = 0.5 * kPi;
  double re = 0.0, im = 0.0;
  for (int b = 0; b + 1 < nb; ++b) {
    const double lo = bp[b], hi = bp[b + 1];
    if (hi - lo < 1e-15) continue;
    const double half = 0.5 * (hi - lo);
    for (int k = -kTsHalfIn; k <= kTsHalfIn; ++k) {
      const double u = k * kTsStepIn;
      const double q = 0.5 * kPi * sinh(u);
      const double ch = cosh(q);
      const double wt = kTsStepIn * 0.5 * kPi * cosh(u) / (ch * ch);
      const double e = 2.0 / (1.0 + exp(2.0 * fabs(q)));
      const double t2 = q >= 0.0 ? hi - half * e : lo + half * e;
      if (!(t2 > lo && t2 < hi)) continue;
      const double st = sin(t2);
      const double A3 = r3 * r3 * (X - st * st / (r2 * r2));
      if (A3 == 0.0) continue;
      double T2 = 1.0;
      for (int j = 0; j < p.tpow; ++j) T2 *= 1.0 - 0.5 * st * st;
      const Cplx J = k2n_over_a(A3, s, p.tpow, i3);
      const double f = half * wt * T2 * cos(2.0 * i2 * t2);
      re += f * J.re;
      im += f * J.im;
    }
  }
  const double pre = 2.0 * r3 * r3 * X;
  return Cplx{pre * re, pre * im};
}

// Re[(i / sigma1) Shat(kh + nu pi) I e^{i ph kh}]; with force = true the
// self-force weight Shat_g(kh) replaces the phase factor
__device__ inline double integrand(const KsParams &p, double kh, int nu, double ph, bool force) {
  const double s1 = sigma1b(p, kh);  // i / [k]_B1
  if (s1 == 0.0) return 0.0;
  const double A = a_of(p, kh, nu);
  const double sv = sin(2.0 * p.beta * (kh + nu * kPi) / p.kappa);
  const double sg = sv > 0.0 ? 1.0 : (sv < 0.0 ? -1.0 : 0.0);
  double ir, ii;
  k2_integral(A, sg, p.tpow, ir, ii);
  const double w = shat(kh + nu * kPi, p.order) / s1;
  // (i / s1) * (ir + i ii) = (-ii + i ir) / s1
  const double vr = -ii * w, vi = ir * w;
  if (force) return vr * shat(kh, p.gather_order);
  return vr * cos(ph * kh) - vi * sin(ph * kh);
}

// One workgroup per output point: sum over panels x tanh-sinh nodes in FP64.
__global__ __launch_bounds__(256) void k_kspace(KsParams p, const Panel *panels, int npanels, const double *phase,
                                                int force, double *out) {
  const double ph = phase[blockIdx.x];
  const int per = 2 * kTsHalf + 1;
  const long long total = (long long)npanels * per;
  double acc = 0.0;
  for (long long t = threadIdx.x; t < total; t += blockDim.x) {
    const Panel pn = panels[t / per];
    const int k = (int)(t % per) - kTsHalf;
    const double u = k * kTsStep;
    const double q = 0.5 * kPi * sinh(u);
    const double ch = cosh(q);
    const double wt = kTsStep * 0.5 * kPi * cosh(u) / (ch * ch);  // d tanh(q)/du * step
    const double half = 0.5 * (pn.b - pn.a);
    // distance from the nearer panel end, without cancellation: 1 - tanh|q| = 2 / (1 + e^{2|q|})
    const double e = 2.0 / (1.0 + exp(2.0 * fabs(q)));
    const double x = q >= 0.0 ? pn.b - half * e : pn.a + half * e;
    if (!(x > pn.a && x < pn.b)) continue;
    acc += half * wt * integrand(p, x, pn.nu, ph, force != 0);
  }
  __shared__ double part[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = -(part[0] + part[1] + part[2] + part[3]) / (2.0 * kPi * kPi * p.r);
}

// One point of relpic_kspace_field: phase 2 i1' + 1 and the transverse nodes
struct KsPoint {
  double ph;
  int i2, i3;
};

// 2D off axis and 3D: one workgroup per output point
__global__ __launch_bounds__(256) void k_kspace_field(KsParams p, const Panel *panels, int npanels,
                                                      const KsPoint *pts, int ndim, double *out) {
  const KsPoint pt = pts[blockIdx.x];
  const int per = 2 * kTsHalf + 1;
  const long long total = (long long)npanels * per;
  double acc = 0.0;
  for (long long t = threadIdx.x; t < total; t += blockDim.x) {
    const Panel pn = panels[t / per];
    const int k = (int)(t % per) - kTsHalf;
    const double u = k * kTsStep;
    const double q = 0.5 * kPi * sinh(u);
    const double ch = cosh(q);
    const double wt = kTsStep * 0.5 * kPi * cosh(u) / (ch * ch);
    const double half = 0.5 * (pn.b - pn.a);
    const double e = 2.0 / (1.0 + exp(2.0 * fabs(q)));
    const double kh = q >= 0.0 ? pn.b - half * e : pn.a + half * e;
    if (!(kh > pn.a && kh < pn.b)) continue;
    const double sB = sigma1b(p, kh);
    if (sB == 0.0) continue;
    const double sv = sin(2.0 * p.beta * (kh + pn.nu * kPi) / p.kappa);
    const double sg = sv > 0.0 ? 1.0 : (sv < 0.0 ? -1.0 : 0.0);
    Cplx I;
    if (ndim == 3) {
      const double X = a_of(p, kh, pn.nu) / (p.r * p.r);
      I = i3_integral(p, X, sg, pt.i2, pt.i3);
    } else {
      const double A = a_of(p, kh, pn.nu);
      const Cplx J = k2n_over_a(A, sg, p.tpow, pt.i2);
      I = Cplx{A * J.re, A * J.im};
    }
    const double w = shat(kh + pn.nu * kPi, p.order) / sB;
    const double vr = -I.im * w, vi = I.re * w;  // (i / sB) I Shat
    acc += half * wt * (vr * cos(pt.ph * kh) - vi * sin(pt.ph * kh));
  }
  __shared__ double part[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double tot = part[0] + part[1] + part[2] + part[3];
    out[blockIdx.x] = ndim == 3 ? -tot / (2.0 * kPi * kPi * kPi * p.r * p.r3) : -tot / (2.0 * kPi * kPi * p.r);
  }
}

// A fixed-capacity list (no heap allocation): panel breakpoints and panels
// are built the same way for the allocating and the allocation-free entry
// points, so both integrate over identical panels.
template <typename T, int CAP>
struct FixedList {
  T v[CAP];
  int n = 0;
  bool overflow = false;
  void push(const T &x) {
    if (n < CAP)
      v[n++] = x;
    else
      overflow = true;
  }
};

// roots of f on [lo, hi] by a uniform scan and bisection
template <typename F, typename L>
void roots(F f, double lo, double hi, int n, L &out) {
  double xa = lo, fa = f(lo);
  for (int i = 1; i <= n; ++i) {
    const double xb = lo + (hi - lo) * i / n;
    const double fb = f(xb);
    if (fa == 0.0) {
      out.push(xa);
    } else if (fa * fb < 0.0) {
      double a = xa, b = xb, va = fa;
      for (int it = 0; it < 200 && b - a > 1e-16; ++it) {
        const double m = 0.5 * (a + b), vm = f(m);
        if (vm == 0.0) {
          a = b = m;
          break;
        }
        if ((vm < 0.0) == (va < 0.0)) {
          a = m;
          va = vm;
        } else {
          b = m;
        }
      }
      out.push(0.5 * (a + b));
    }
    xa = xb;
    fa = fb;
  }
}

constexpr int kMaxBreaks = 256;  // breakpoints of one zone

// Panels between consecutive breakpoints (A = 0, A = 1, sin(beta k1' dt) = 0,
// the zone edges and 0) of every zone nu = -nu_max .. nu_max, written to out;
// false if more than cap panels (or breakpoints) are needed.
// In 3D the levels of A = r2^2 X where the theta2 integrand changes form:
// X = 0, 1/r3^2, 1/r2^2, 1/r2^2 + 1/r3^2.
template <typename L>
bool make_panels_into(const KsParams &p, int nu_max, L &out, int ndim = 2) {
  const double lo = -0.5 * kPi, hi = 0.5 * kPi;
  const double q23 = ndim == 3 ? p.r * p.r / (p.r3 * p.r3) : 0.0;
  const double lev3[4] = {0.0, q23, 1.0, 1.0 + q23};
  const double lev2[2] = {0.0, 1.0};
  const double *levels = ndim == 3 ? lev3 : lev2;
  const int nlev = ndim == 3 ? 4 : 2;
  for (int nu = -nu_max; nu <= nu_max; ++nu) {
    FixedList<double, kMaxBreaks> bp;
    bp.push(lo);
    bp.push(0.0);
    bp.push(hi);
    for (int li = 0; li < nlev; ++li) {
      const double lev = levels[li];
      roots([&](double k) { return a_of(p, k, nu) - lev; }, lo, hi, 4000, bp);
    }
    roots([&](double k) { return std::sin(2.0 * p.beta * (k + nu * kPi) / p.kappa); }, lo, hi, 4000, bp);
    if (bp.overflow) return false;
    std::sort(bp.v, bp.v + bp.n);
    for (int i = 0; i + 1 < bp.n; ++i) {
      const double a = std::max(lo, bp.v[i]), b = std::min(hi, bp.v[i + 1]);
      if (b - a > 1e-14) out.push(Panel{a, b, nu, 0});
    }
  }
  return !out.overflow;
}

struct PanelVec {
  std::vector<Panel> v;
  bool overflow = false;
  void push(const Panel &x) { v.push_back(x); }
};

std::vector<Panel> make_panels(const KsParams &p, int nu_max, int ndim = 2) {
  PanelVec out;
  make_panels_into(p, nu_max, out, ndim);
  return out.v;
}


// ---- allocation-free variant --------------------------------------------------------
// Device scratch for relpic_kspace_e1_noalloc: panels, point phases and the
// per-point results.  Each GPU the library runs on holds its own copy until
// the process ends; its device address is looked up once per device.
constexpr int kNaMaxPanels = 1024;
constexpr int kNaMaxPoints = 4096;
constexpr size_t kNaPanelBytes = sizeof(Panel) * kNaMaxPanels;       // 24 KiB
constexpr size_t kNaPhaseOff = (kNaPanelBytes + 255) & ~size_t(255);
constexpr size_t kNaOutOff = kNaPhaseOff + sizeof(double) * kNaMaxPoints;
constexpr size_t kNaBytes = kNaOutOff + sizeof(double) * kNaMaxPoints;  // 88 KiB in all
static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mutex;
void *g_na_ptr[kNaMaxDevices] = {};

// device address of `scratch` on the current device (hipGetSymbolAddress,
// once per device); the array's host-side name is not a device address
relpic_status scratch_ptr(int dev, unsigned char **out) {
  if (dev < 0 || dev >= kNaMaxDevices) return fail_noalloc(RELPIC_EINVAL, "kspace_e1_noalloc", "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_na_mutex);
  if (!g_na_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail_noalloc(RELPIC_EDEVICE, "kspace_e1_noalloc", "hipGetSymbolAddress failed");
    g_na_ptr[dev] = ptr;
  }
  *out = (unsigned char *)g_na_ptr[dev];
  return RELPIC_OK;
}

relpic_status check_params(const relpic_kspace *q, KsParams &p) {
  if (!q) return fail(RELPIC_EINVAL, "kspace: null parameters");
  if (q->M < 1 || q->M > kKsMaxM || (q->M > 1 && !q->C)) return fail(RELPIC_EINVAL, "kspace: bad axial operator");
  if (!(q->kappa > 1.0) || !(q->r > 0.0) || !(q->beta > 0.0 && q->beta <= 1.0))
    return fail(RELPIC_EINVAL, "kspace: need kappa > 1, r > 0, 0 < beta <= 1");
  if (q->shape_order < 0 || q->shape_order > 4 || q->tpow < 0 || q->tpow > 2 || q->nu_max < 0 || q->nu_max > 8)
    return fail(RELPIC_EINVAL, "kspace: bad shape order, transverse factor power or zone count");
  if (q->MB < 0 || q->MB > kKsMaxM || (q->MB > 1 && !q->CB)) return fail(RELPIC_EINVAL, "kspace: bad operator on B");
  std::memset(&p, 0, sizeof(p));
  p.M = std::max(q->M, q->MB);
  for (int l = 0; l < q->M; ++l) p.C[l] = q->M == 1 && !q->C ? 1.0 : q->C[l];
  for (int l = 0; l < p.M; ++l) p.CB[l] = q->MB == 0 ? p.C[l] : (l < q->MB ? (q->CB ? q->CB[l] : 1.0) : 0.0);
  p.kappa = q->kappa;
  p.r = q->r;
  p.beta = q->beta;
  p.order = q->shape_order;
  p.tpow = q->tpow;
  p.gather_order = q->shape_order;
  return RELPIC_OK;
}

relpic_status run(const KsParams &p, int nu_max, const relpic_device *dev, const std::vector<double> &phase,
                  int force, double *out) {
  const std::vector<Panel> panels = make_panels(p, nu_max);
  const int dv = dev ? dev->device : 0;
  HIP_OK(hipSetDevice(dv));
  hipStream_t st = dev ? (hipStream_t)dev->stream : nullptr;
  auto dalloc = [&](size_t bytes) -> void * {
    void *ptr = nullptr;
    if (dev && dev->alloc)
      ptr = dev->alloc(bytes, dev->user);
    else if (hipMalloc(&ptr, bytes) != hipSuccess)
      ptr = nullptr;
    return ptr;
  };
  auto dfree = [&](void *ptr) {
    if (!ptr) return;
    if (dev && dev->free)
      dev->free(ptr, dev->user);
    else if (!(dev && dev->alloc))
      (void)hipFree(ptr);
  };
  Panel *dp = (Panel *)dalloc(sizeof(Panel) * panels.size());
  double *dph = (double *)dalloc(sizeof(double) * phase.size());
  double *dout = (double *)dalloc(sizeof(double) * phase.size());
  relpic_status rc = RELPIC_OK;
  if (!dp || !dph || !dout) {
    rc = fail(RELPIC_ENOMEM, "kspace: allocation failed");
  } else {
    hipError_t e = hipMemcpyAsync(dp, panels.data(), sizeof(Panel) * panels.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dph, phase.data(), sizeof(double) * phase.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      k_kspace<<<(unsigned)phase.size(), 256, 0, st>>>(p, dp, (int)panels.size(), dph, force, dout);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(out, dout, sizeof(double) * phase.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(RELPIC_EDEVICE, std::string("kspace: ") + hipGetErrorString(e));
  }
  dfree(dp);
  dfree(dph);
  dfree(dout);
  return rc;
}

}  // namespace

extern "C" {

relpic_status relpic_kspace_e1(const relpic_kspace *q, const relpic_device *dev, int64_t npts, const double *i1_rel,
                               double *out) {
  return guarded("kspace_e1", [&]() -> relpic_status {
    KsParams p;
    if (relpic_status e = check_params(q, p)) return e;
    if (npts < 1 || npts > (1 << 20) || !i1_rel || !out) return fail(RELPIC_EINVAL, "kspace_e1: bad points");
    std::vector<double> phase(npts);
    for (int64_t i = 0; i < npts; ++i) {
      if (!std::isfinite(i1_rel[i]) || std::fabs(i1_rel[i]) > 1e6) return fail(RELPIC_EINVAL, "kspace_e1: bad index");
      phase[i] = 2.0 * i1_rel[i] + 1.0;
    }
    return run(p, q->nu_max, dev, phase, 0, out);
  });
}

relpic_status relpic_kspace_self_force(const relpic_kspace *q, const relpic_device *dev, int gather_order,
                                       double *out) {
  return guarded("kspace_self_force", [&]() -> relpic_status {
    KsParams p;
    if (relpic_status e = check_params(q, p)) return e;
    if (!out || gather_order < 0 || gather_order > 4) return fail(RELPIC_EINVAL, "kspace_self_force: bad arguments");
    p.gather_order = gather_order;
    std::vector<double> phase(1, 0.0);
    return run(p, q->nu_max, dev, phase, 1, out);
  });
}

relpic_status relpic_kspace_field(const relpic_kspace *q, const relpic_device *dev, int ndim, double r3, int64_t npts,
                                  const double *i1_rel, const int32_t *i2, const int32_t *i3, double *out) {
  return guarded("kspace_field", [&]() -> relpic_status {
    KsParams p;
    if (relpic_status e = check_params(q, p)) return e;
    if (ndim != 2 && ndim != 3) return fail(RELPIC_EINVAL, "kspace_field: ndim must be 2 or 3");
    if (ndim == 3 && !(r3 > 0.0)) return fail(RELPIC_EINVAL, "kspace_field: need r3 > 0");
    if (npts < 1 || npts > (1 << 20) || !i1_rel || !i2 || (ndim == 3 && !i3) || !out)
      return fail(RELPIC_EINVAL, "kspace_field: bad points");
    p.r3 = ndim == 3 ? r3 : 1.0;
    std::vector<KsPoint> pts((size_t)npts);
    for (int64_t i = 0; i < npts; ++i) {
      if (!std::isfinite(i1_rel[i]) || std::fabs(i1_rel[i]) > 1e6 || std::abs(i2[i]) > 100000 ||
          (ndim == 3 && std::abs(i3[i]) > 100000))
        return fail(RELPIC_EINVAL, "kspace_field: bad index");
      pts[i] = KsPoint{2.0 * i1_rel[i] + 1.0, i2[i], ndim == 3 ? i3[i] : 0};
    }
    const std::vector<Panel> panels = make_panels(p, q->nu_max, ndim);
    const int dv = dev ? dev->device : 0;
    HIP_OK(hipSetDevice(dv));
    hipStream_t st = dev ? (hipStream_t)dev->stream : nullptr;
    auto dalloc = [&](size_t bytes) -> void * {
      void *ptr = nullptr;
      if (dev && dev->alloc)
        ptr = dev->alloc(bytes, dev->user);
      else if (hipMalloc(&ptr, bytes) != hipSuccess)
        ptr = nullptr;
      return ptr;
    };
    auto dfree = [&](void *ptr) {
      if (!ptr) return;
      if (dev && dev->free)
        dev->free(ptr, dev->user);
      else if (!(dev && dev->alloc))
        (void)hipFree(ptr);
    };
    Panel *dp = (Panel *)dalloc(sizeof(Panel) * panels.size());
    KsPoint *dpt = (KsPoint *)dalloc(sizeof(KsPoint) * pts.size());
    double *dout = (double *)dalloc(sizeof(double) * pts.size());
    relpic_status rc = RELPIC_OK;
    if (!dp || !dpt || !dout) {
      rc = fail(RELPIC_ENOMEM, "kspace_field: allocation failed");
    } else {
      hipError_t e = hipMemcpyAsync(dp, panels.data(), sizeof(Panel) * panels.size(), hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dpt, pts.data(), sizeof(KsPoint) * pts.size(), hipMemcpyHostToDevice, st);
      if (e == hipSuccess) {
        k_kspace_field<<<(unsigned)pts.size(), 256, 0, st>>>(p, dp, (int)panels.size(), dpt, ndim, dout);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(double) * pts.size(), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) rc = fail(RELPIC_EDEVICE, std::string("kspace_field: ") + hipGetErrorString(e));
    }
    dfree(dp);
    dfree(dpt);
    dfree(dout);
    return rc;
  });
}

relpic_status relpic_kspace_e1_noalloc(const relpic_kspace *q, const relpic_device *dev, int64_t npts,
                                       const double *i1_rel, double *out) {
  return guarded("kspace_e1_noalloc", [&]() -> relpic_status {
    KsParams p;
    if (relpic_status e = check_params(q, p)) return e;
    if (npts < 1 || npts > kNaMaxPoints || !i1_rel || !out)
      return fail_noalloc(RELPIC_EINVAL, "kspace_e1_noalloc", "need 1 <= npts <= 4096 and non-null arrays");
    if (dev && (dev->alloc || dev->free))
      return fail_noalloc(RELPIC_EINVAL, "kspace_e1_noalloc", "allocator callbacks are not used here: pass none");
    double phase[kNaMaxPoints];
    for (int64_t i = 0; i < npts; ++i) {
      if (!std::isfinite(i1_rel[i]) || std::fabs(i1_rel[i]) > 1e6)
        return fail_noalloc(RELPIC_EINVAL, "kspace_e1_noalloc", "bad index");
      phase[i] = 2.0 * i1_rel[i] + 1.0;
    }
    FixedList<Panel, kNaMaxPanels> panels;  // on the stack (24 KiB): no heap allocation
    if (!make_panels_into(p, q->nu_max, panels))
      return fail_noalloc(RELPIC_ERANGE, "kspace_e1_noalloc", "more than 1024 quadrature panels: lower nu_max");
    const int dv = dev ? dev->device : 0;
    HIP_OK(hipSetDevice(dv));
    hipStream_t st = dev ? (hipStream_t)dev->stream : nullptr;
    unsigned char *base = nullptr;
    if (relpic_status e = scratch_ptr(dv, &base)) return e;
    Panel *dp = (Panel *)base;
    double *dph = (double *)(base + kNaPhaseOff);
    double *dout = (double *)(base + kNaOutOff);
    HIP_OK(hipMemcpyAsync(dp, panels.v, sizeof(Panel) * panels.n, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(dph, phase, sizeof(double) * npts, hipMemcpyHostToDevice, st));
    k_kspace<<<(unsigned)npts, 256, 0, st>>>(p, dp, panels.n, dph, 0, dout);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(out, dout, sizeof(double) * npts, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    return RELPIC_OK;
  });
}

}  // extern "C"
