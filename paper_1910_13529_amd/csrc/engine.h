// Host-side state of one relpic simulation, shared by the C ABI and the
// batched engine (internal to relpic).
#pragma once

#include <hip/hip_runtime.h>

#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/relpic.h"
#include "kernels.h"

namespace relpic_host {

struct Species {
  double qm = -1.0, Q = -1.0;
  long long cap = 0, n = 0;
  int *cell = nullptr;
  void *o[3] = {nullptr, nullptr, nullptr};
  void *u[3] = {nullptr, nullptr, nullptr};
  int *id = nullptr;
  long long next_id = 0;
  // second buffers for the sort (swapped after each sort)
  int *cell2 = nullptr;
  void *o2[3] = {nullptr, nullptr, nullptr};
  void *u2[3] = {nullptr, nullptr, nullptr};
  int *id2 = nullptr;
  unsigned *keys = nullptr, *keys2 = nullptr, *idx = nullptr, *idx2 = nullptr;
  void *sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  bool dirty = true;   // needs a sort before the next step
  long long sorted_at = 0;  // step of the last sort
  int K = 1;           // particles per thread in the push kernel
  bool tile_keys = false;  // sort key order: 3D tiles (sparse) or rows (dense)
  bool long_runs = false;  // tile order and runs of several particles per cell
  // index ranges of the sort tiles after the last tile sort (push chunks)
  int *tile_first = nullptr, *tile_end = nullptr;
  long long tiles_cap = 0, ntiles = 0, n_tiled = 0;
  bool inject = false;
  int ppc[3] = {1, 1, 1};
  double uth = 0.0;
  unsigned long long seed = 0, inj_count = 0;
};

relpic_status fail(relpic_status s, const std::string &msg);
// does not allocate: usable while handling std::bad_alloc
relpic_status fail_noalloc(relpic_status s, const char *where, const char *what) noexcept;

// Every extern "C" entry point runs its body through guarded(): a C++
// exception (a host allocation that fails, a container length error) is
// turned into a status and a message instead of crossing the C boundary.
template <typename F>
relpic_status guarded(const char *where, F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return fail_noalloc(RELPIC_ENOMEM, where, "host allocation failed");
  } catch (const std::length_error &) {
    return fail_noalloc(RELPIC_ENOMEM, where, "host buffer size out of range");
  } catch (const std::exception &e) {
    return fail_noalloc(RELPIC_EINVAL, where, e.what());
  } catch (...) {
    return fail_noalloc(RELPIC_EINVAL, where, "unexpected C++ exception");
  }
}

}  // namespace relpic_host

using relpic_host::Species;

struct relpic_sim {
  relpic_grid grid{};
  int ndim = 2;
  int n[3] = {1, 1, 1};
  double dx[3] = {1, 1, 1};
  relpic_precision prec = RELPIC_FP64;
  size_t esz = 8;
  int M = 1;                        // stencil half-width of both axial operators (the shorter one zero-padded)
  double C[relpic::kMaxM] = {1.0};   // d+ (E -> B): [k]_E1
  double CB[relpic::kMaxM] = {1.0};  // d- (B -> E, Gauss, continuity): [k]_B1
  bool correct = false;              // J1 correction on (d- wider than two points)
  relpic_device dev{};
  hipStream_t st = nullptr;
  long long N = 0;
  void *F[10] = {};  // E1 E2 E3 B1 B2 B3 J1 J2 J3 J1c; B holds B^n between calls
  void *Bx[3] = {};  // second B buffer (B at the other half-integer time inside a call)
  void *Ex[3] = {};  // second E buffer for the fused update (3D grids that qualify)
  bool fuse = false; // fused E and B update in use
  relpic::JBox *jbox = nullptr;  // two deposit boxes, alternating by step parity
  relpic::JBox *blockbox = nullptr;  // per-workgroup deposit boxes of the push kernel
  long long blockbox_n = 0;
  void *taps = nullptr;
  int ng = 0;
  int filt_npass = 0;      // current filter: binomial passes along x1 (0: off)
  double filt_comp = 0.0;  // and the compensator's c: (-c/4, 1 + c/2, -c/4)
  std::vector<Species> sp;
  long long step = 0, ws = 0;
  long long sort_interval = 25;  // re-sort every this many steps (0: only after loads)
  int *err = nullptr;
  double *dbuf = nullptr;      // diagnostics accumulators (8 doubles)
  // counting sort of the particle keys: bucket counts and scan scratch
  unsigned *kcount = nullptr;
  unsigned long long *kbsum = nullptr;
  unsigned *kbocc = nullptr;
  long long kcount_cap = 0, kblocks_cap = 0;
  double *rho = nullptr;       // FP64 scratch for the Gauss diagnostic
  double *rho_bg = nullptr;    // background charge, storage layout
  double *gather_buf = nullptr;  // FP64 staging of fields gathered at particles (diagnostic)
  long long gather_cap = 0;      // its capacity in particles
  std::vector<void *> owned;
  // per-kernel event timing
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  // (class + 64 * (species + 1) for a species' push, class otherwise; index of the start event)
  std::vector<std::pair<int, size_t>> ev_marks;
};

#define HIP_OK(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return relpic_host::fail(RELPIC_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

namespace relpic_host {

using namespace relpic;

void *dev_alloc(relpic_sim *s, size_t bytes);
void dev_release(relpic_sim *s, void *p);
void dev_free_all(relpic_sim *s);

inline Geo make_geo(const relpic_sim *s) {
  Geo g{};
  g.n1 = s->n[0];
  g.n2 = s->n[1];
  g.n3 = s->n[2];
  g.window = s->grid.bc1 == RELPIC_BC_WINDOW ? 1 : 0;
  g.ws_mod = (int)(((s->ws % s->n[0]) + s->n[0]) % s->n[0]);
  g.N = s->N;
  g.dv1 = make_fastdiv((unsigned)g.n1);
  g.dv2 = make_fastdiv((unsigned)g.n2);
  return g;
}

template <typename Real>
inline Fields<Real> fields(const relpic_sim *s) {
  Fields<Real> f;
  f.E1 = (Real *)s->F[0];
  f.E2 = (Real *)s->F[1];
  f.E3 = (Real *)s->F[2];
  f.B1 = (Real *)s->F[3];
  f.B2 = (Real *)s->F[4];
  f.B3 = (Real *)s->F[5];
  f.J1 = (Real *)s->F[6];
  f.J2 = (Real *)s->F[7];
  f.J3 = (Real *)s->F[8];
  f.J1c = (Real *)s->F[9];
  return f;
}

template <typename Real>
inline Particles<Real> parts(const Species &sp) {
  Particles<Real> p;
  p.cell = sp.cell;
  p.o1 = (Real *)sp.o[0];
  p.o2 = (Real *)sp.o[1];
  p.o3 = (Real *)sp.o[2];
  p.u1 = (Real *)sp.u[0];
  p.u2 = (Real *)sp.u[1];
  p.u3 = (Real *)sp.u[2];
  p.n = sp.n;
  return p;
}

inline double cell_volume(const relpic_sim *s) {
  double v = 1.0;
  for (int d = 0; d < s->ndim; ++d) v *= s->dx[d];
  return v;
}

// axial coefficients C_l c / dx1 of the operator on E (d+, E -> B; c: the
// time factor of the update)
template <typename Real>
inline Axial<Real> axial_scaled(const relpic_sim *s, double c) {
  Axial<Real> ax{};
  ax.M = s->M;
  for (int l = 0; l < s->M; ++l) ax.c[l] = (Real)(s->C[l] * c / s->dx[0]);
  return ax;
}

// the same for the operator on B (d-, B -> E)
template <typename Real>
inline Axial<Real> axial_scaled_b(const relpic_sim *s, double c) {
  Axial<Real> ax{};
  ax.M = s->M;
  for (int l = 0; l < s->M; ++l) ax.c[l] = (Real)(s->CB[l] * c / s->dx[0]);
  return ax;
}

// push constants of one species for one step (shift: the window advances
// after the step)
template <typename Real>
inline PushParams<Real> push_params(const relpic_sim *s, const Species &sp, int shift) {
  const double dt = s->grid.dt, dV = cell_volume(s);
  PushParams<Real> q{};
  q.half_qmdt = (Real)(0.5 * sp.qm * dt);
  for (int d = 0; d < 3; ++d) q.dtdx[d] = (Real)(d < s->ndim ? dt / s->dx[d] : 0.0);
  q.f1 = (Real)(-sp.Q * s->dx[0] / (dV * dt));
  q.f2 = (Real)(-sp.Q * s->dx[1] / (dV * dt));
  q.f3 = (Real)(s->ndim == 3 ? -sp.Q * s->dx[2] / (dV * dt) : 0.0);
  q.fv = (Real)(sp.Q / dV);
  q.shift = shift;
  return q;
}

}  // namespace relpic_host
