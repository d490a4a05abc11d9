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
template <typename L>
bool make_panels_into(const KsParams &p, int nu_max, L &out) {
  const double lo = -0.5 * kPi, hi = 0.5 * kPi;
  for (int nu = -nu_max; nu <= nu_max; ++nu) {
    FixedList<double, kMaxBreaks> bp;
    bp.push(lo);
    bp.push(0.0);
    bp.push(hi);
    for (double lev : {0.0, 1.0}) roots([&](double k) { return a_of(p, k, nu) - lev; }, lo, hi, 4000, bp);
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

std::vector<Panel> make_panels(const KsParams &p, int nu_max) {
  PanelVec out;
  make_panels_into(p, nu_max, out);
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
