// Adjoint engine and its C ABI: gradient of a field loss with respect to the
// axial coefficients C_l of the customized solver, by reverse-mode
// differentiation of the field advance and the J1 correction with time-step
// checkpoints.
//
// Forward (2D periodic grid, fields zero at t = 0, ballistic particles whose
// current does not depend on C; b_n = B^{n-1/2}, e_n = E^n):
//   b_{n+1} = b_n - dt curl+ e_n
//   e_{n+1} = e_n + dt curl- b_{n+1} - dt G J^{n+1/2}     (G = 1 for Yee)
//   L = sum_{n=1..N} l_n(e_n, (b_n + b_{n+1}) / 2)
// Reverse, for n = N .. 1, with adjoint fields eA (of e) and bA (of b):
//   bA += (1/2) dl_n/dB                         -> complete adjoint of b_{n+1}
//   dC += -dt <bA, dcurl+/dC e_n>
//   eA += dl_n/dE;  eA -= dt curl- bA           -> complete adjoint of e_n
//   dC += dt <eA, dcurl-/dC b_n> + dt <eA1, G S_l G J1_{n-1}>
//   bA += dt curl+ eA + (1/2) dl_n/dB           -> adjoint of b_n (less l_{n-1}'s part)
// using (curl+)^T = curl-, dG/dC_l = -G S_l G with S_l the (2l - 1)-point box
// sum (the telescoped stencil K has K_m = sum_{l > |m|} C_l), and symmetric
// G.  Fields (e_n, b_n) are checkpointed every `every` steps; the backward
// pass recomputes each segment from its checkpoint, storing its steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "adjoint_kernels.h"
#include "engine.h"
#include "solver_setup.h"

using namespace relpic;
using namespace relpic_host;

struct relpic_adj {
  relpic_sim *s = nullptr;
  long long nsteps = 0;
  int every = 20;
  relpic_loss_box box{};
  int M = 1;
  int nparts = 0;
  bool forward_done = false;
  std::vector<double> C;
  void *p0[6] = {};        // initial particle state (cell, o1, o2, u1, u2, u3)
  void *ckF = nullptr;     // checkpoints: nck x 6 field arrays (e, b)
  void *ckP = nullptr;     // checkpoints of the particle state: nck x 6 arrays
  void *segF = nullptr;    // segment storage: (every + 2) x 6 field arrays
  void *segJ = nullptr;    // segment J1c: every arrays
  JBox *segbox = nullptr;  // segment deposit boxes
  void *aE[3] = {}, *aB[3] = {};
  double *dacc = nullptr;  // [0] loss, [1 .. M] dL/dC
};

namespace {

relpic_status check_adj(relpic_adj *a) {
  if (!a || !a->s) return fail(RELPIC_EINVAL, "null adjoint handle");
  return RELPIC_OK;
}

size_t particle_bytes(const relpic_sim *s, int k) { return k == 0 ? sizeof(int) : s->esz; }

void *particle_array(Species &sp, int k) {
  switch (k) {
    case 0: return sp.cell;
    case 1: return sp.o[0];
    case 2: return sp.o[1];
    case 3: return sp.u[0];
    case 4: return sp.u[1];
    default: return sp.u[2];
  }
}

// copy the particle state to (dir = 0) or from (dir = 1) six arrays at dst
relpic_status particles_copy(relpic_adj *a, void *const *arrs, int dir) {
  relpic_sim *s = a->s;
  if (s->sp.empty()) return RELPIC_OK;
  Species &sp = s->sp[0];
  for (int k = 0; k < 6; ++k) {
    const size_t bytes = particle_bytes(s, k) * (size_t)a->nparts;
    if (!bytes) continue;
    if (dir == 0)
      HIP_OK(hipMemcpyAsync(arrs[k], particle_array(sp, k), bytes, hipMemcpyDeviceToDevice, s->st));
    else
      HIP_OK(hipMemcpyAsync(particle_array(sp, k), arrs[k], bytes, hipMemcpyDeviceToDevice, s->st));
  }
  return RELPIC_OK;
}

void *slot_ptr(void *base, size_t slot_bytes, long long k) { return (char *)base + slot_bytes * k; }

template <typename Real>
struct Ctx {
  relpic_adj *a;
  relpic_sim *s;
  Geo g;
  size_t fb;  // bytes of one field array
  Real *E[3];
  Real *bc[3], *bn[3];  // b_n and b_{n+1}
  double dt, w;
  Ctx(relpic_adj *a_) : a(a_), s(a_->s) {
    g = make_geo(s);
    fb = s->esz * (size_t)s->N;
    for (int d = 0; d < 3; ++d) {
      E[d] = (Real *)s->F[d];
      bc[d] = (Real *)s->F[3 + d];
      bn[d] = (Real *)s->Bx[d];
    }
    dt = s->grid.dt;
    w = s->dx[0] * s->dx[1] * dt;
  }
  LossBox loss_box(long long n) const {
    LossBox b;
    b.c1 = a->box.x1 + a->box.v1 * n * dt;
    b.c2 = a->box.x2;
    b.h1 = a->box.half1;
    b.h2 = a->box.half2;
    b.dx1 = s->dx[0];
    b.dx2 = s->dx[1];
    return b;
  }
  Fields<Real> fields_with(Real *const Ee[3], Real *const Bb[3]) const {
    Fields<Real> f = fields<Real>(s);
    f.E1 = Ee[0];
    f.E2 = Ee[1];
    f.E3 = Ee[2];
    f.B1 = Bb[0];
    f.B2 = Bb[1];
    f.B3 = Bb[2];
    return f;
  }
  // Bout = Bin - c curl+ Ee
  void curl_plus(Real *const Ee[3], Real *const Bin[3], Real *const Bout[3], double c) const {
    const Fields<Real> f = fields_with(Ee, Bin);
    launch_curl_e<Real>(2, g, f, Bin, Bout, axial_scaled<Real>(s, c), (Real)(c / s->dx[1]), Real(0), s->st);
  }
  // Ee += c curl- Bb
  void curl_minus(Real *const Ee[3], Real *const Bb[3], double c) const {
    const Fields<Real> f = fields_with(Ee, Bb);
    launch_curl_b<Real>(2, g, f, axial_scaled_b<Real>(s, c), (Real)(c / s->dx[1]), Real(0), s->st);
  }
  // particle phase and E update of step n: e_{n+1} = e_n + dt curl- b_{n+1} - dt G J.
  // jbox receives the deposit box; J1c (M > 1) is left in F[9].
  relpic_status advance_e(long long n) {
    JBox *box = s->jbox + (n & 1);
    JBox *next = s->jbox + ((n + 1) & 1);
    if (!s->sp.empty() && a->nparts > 0) {
      Species &sp = s->sp[0];
      PushChunks pc;  // runs of 256 K particles in array order
      pc.K = sp.K;
      const long long nb = push_grid(pc, sp.n);
      if (nb > s->blockbox_n) {
        s->blockbox = (JBox *)dev_alloc(s, sizeof(JBox) * (size_t)nb);
        if (!s->blockbox) return fail(RELPIC_ENOMEM, "adjoint: allocation of workgroup boxes failed");
        s->blockbox_n = nb;
      }
      const Fields<Real> f = fields_with(E, bn);
      const HalfB<Real> Bh{bc[0], bc[1], bc[2]};
      launch_push_deposit<Real>(2, g, f, Bh, parts<Real>(sp), push_params<Real>(s, sp, 0), pc, false, false,
                                s->blockbox, s->err, s->st);
      launch_merge_boxes(s->blockbox, nb, box, s->st);
    }
    const Fields<Real> f = fields_with(E, bn);
    const Real *J1src = f.J1;
    if (s->M > 1) {
      launch_jcorr<Real>(g, f.J1, f.J1c, (const Real *)s->taps, s->ng, box, s->st);
      J1src = f.J1c;
    }
    curl_minus(E, bn, dt);
    launch_add_j<Real>(g, f, J1src, (Real)dt, box, s->M > 1 ? s->ng : 0, next, s->st);
    return RELPIC_OK;
  }
  void swap_b() {
    for (int d = 0; d < 3; ++d) std::swap(bc[d], bn[d]);
  }
};

relpic_status set_coefficients(relpic_adj *a, const double *C) {
  relpic_sim *s = a->s;
  for (int l = 0; l < a->M; ++l)
    if (!std::isfinite(C[l])) return fail(RELPIC_EINVAL, "adjoint: non-finite coefficient");
  const double cn = courant_number(2, s->dx, s->grid.dt, C, a->M);
  if (!(cn < 1.0)) return fail(RELPIC_EUNSTABLE, "adjoint: coefficients violate the Courant limit");
  for (int l = 0; l < a->M; ++l) s->C[l] = s->CB[l] = C[l];  // one operator on E and on B
  s->correct = a->M > 1;
  if (a->M > 1) {
    std::vector<double> taps;
    const double tol = s->prec == RELPIC_FP64 ? 1e-16 : 1e-9;
    if (!correction_taps(C, a->M, tol, kMaxTaps, taps))
      return fail(RELPIC_EINVAL, "adjoint: J1 correction does not converge within the tap limit");
    s->ng = (int)taps.size() - 1;
    std::vector<unsigned char> host(s->esz * taps.size());
    for (size_t i = 0; i < taps.size(); ++i) {
      if (s->esz == 4) {
        const float v = (float)taps[i];
        std::memcpy(&host[i * 4], &v, 4);
      } else {
        std::memcpy(&host[i * 8], &taps[i], 8);
      }
    }
    HIP_OK(hipMemcpyAsync(s->taps, host.data(), host.size(), hipMemcpyHostToDevice, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
  }
  a->C.assign(C, C + a->M);
  return RELPIC_OK;
}

template <typename Real>
relpic_status do_forward(relpic_adj *a, const double *C, double *loss) {
  relpic_sim *s = a->s;
  a->forward_done = false;
  if (relpic_status e = set_coefficients(a, C)) return e;
  Ctx<Real> c(a);
  for (int k = 0; k < 9; ++k) HIP_OK(hipMemsetAsync(s->F[k], 0, c.fb, s->st));
  for (int d = 0; d < 3; ++d) HIP_OK(hipMemsetAsync(s->Bx[d], 0, c.fb, s->st));
  HIP_OK(hipMemsetAsync(a->dacc, 0, sizeof(double) * (1 + kMaxM), s->st));
  launch_reset_box(s->jbox, s->st);
  launch_reset_box(s->jbox + 1, s->st);
  if (relpic_status e = particles_copy(a, a->p0, 1)) return e;
  const long long N = a->nsteps;
  for (long long n = 0; n <= N; ++n) {
    if (n < N && n % a->every == 0) {
      const long long k = n / a->every;
      for (int d = 0; d < 3; ++d) {
        HIP_OK(hipMemcpyAsync(slot_ptr(a->ckF, c.fb, 6 * k + d), c.E[d], c.fb, hipMemcpyDeviceToDevice, s->st));
        HIP_OK(hipMemcpyAsync(slot_ptr(a->ckF, c.fb, 6 * k + 3 + d), c.bc[d], c.fb, hipMemcpyDeviceToDevice, s->st));
      }
      void *arrs[6];
      for (int q = 0; q < 6; ++q) arrs[q] = slot_ptr(a->ckP, 8 * (size_t)a->nparts, 6 * k + q);
      if (relpic_status e = particles_copy(a, arrs, 0)) return e;
    }
    c.curl_plus(c.E, c.bc, c.bn, c.dt);
    if (n >= 1)
      launch_adj_loss<Real>(c.g, c.E[0], c.E[1], c.bc[2], c.bn[2], c.loss_box(n), c.w, a->dacc, s->st);
    if (n == N) break;
    if (relpic_status e = c.advance_e(n)) return e;
    c.swap_b();
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(loss, a->dacc, sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  a->forward_done = true;
  return RELPIC_OK;
}

template <typename Real>
relpic_status do_backward(relpic_adj *a, double *dLdC) {
  relpic_sim *s = a->s;
  Ctx<Real> c(a);
  const int M = a->M;
  const long long N = a->nsteps, S = a->every;
  for (int d = 0; d < 3; ++d) {
    HIP_OK(hipMemsetAsync(a->aE[d], 0, c.fb, s->st));
    HIP_OK(hipMemsetAsync(a->aB[d], 0, c.fb, s->st));
  }
  HIP_OK(hipMemsetAsync(a->dacc, 0, sizeof(double) * (1 + kMaxM), s->st));
  Real *aE[3] = {(Real *)a->aE[0], (Real *)a->aE[1], (Real *)a->aE[2]};
  Real *aB[3] = {(Real *)a->aB[0], (Real *)a->aB[1], (Real *)a->aB[2]};
  double *dC = a->dacc + 1;
  const long long nseg = (N + S - 1) / S;
  auto segE = [&](long long k, int d) { return (Real *)slot_ptr(a->segF, c.fb, 6 * k + d); };
  auto segB = [&](long long k, int d) { return (Real *)slot_ptr(a->segF, c.fb, 6 * k + 3 + d); };
  for (long long seg = nseg - 1; seg >= 0; --seg) {
    const long long c0 = seg * S, c1 = std::min(c0 + S, N);
    // restore the checkpoint of step c0
    for (int d = 0; d < 3; ++d) {
      HIP_OK(hipMemcpyAsync(c.E[d], slot_ptr(a->ckF, c.fb, 6 * seg + d), c.fb, hipMemcpyDeviceToDevice, s->st));
      HIP_OK(hipMemcpyAsync(c.bc[d], slot_ptr(a->ckF, c.fb, 6 * seg + 3 + d), c.fb, hipMemcpyDeviceToDevice, s->st));
    }
    void *arrs[6];
    for (int q = 0; q < 6; ++q) arrs[q] = slot_ptr(a->ckP, 8 * (size_t)a->nparts, 6 * seg + q);
    if (relpic_status e = particles_copy(a, arrs, 1)) return e;
    launch_reset_box(s->jbox + (c0 & 1), s->st);
    // recompute the segment, storing e_n, b_n (n = c0 .. c1), b_{c1+1}, J1c_n and the boxes
    // (one copy launch per step: e_n, b_n, and the box and J1c of step n - 1,
    // which step n's particle phase overwrites)
    for (long long n = c0; n <= c1; ++n) {
      const long long k = n - c0;
      CopyList cl;
      cl.n = 0;
      if (k > 0) {
        cl.op[cl.n++] = CopyOp{a->segbox + (k - 1), s->jbox + ((n - 1) & 1), sizeof(JBox)};
        if (M > 1) cl.op[cl.n++] = CopyOp{slot_ptr(a->segJ, c.fb, k - 1), s->F[9], c.fb};
      }
      for (int d = 0; d < 3; ++d) {
        cl.op[cl.n++] = CopyOp{segE(k, d), c.E[d], c.fb};
        cl.op[cl.n++] = CopyOp{segB(k, d), c.bc[d], c.fb};
      }
      launch_copy_many(cl, s->st);
      c.curl_plus(c.E, c.bc, c.bn, c.dt);
      if (n == c1) {
        cl.n = 0;
        for (int d = 0; d < 3; ++d) cl.op[cl.n++] = CopyOp{segB(k + 1, d), c.bn[d], c.fb};
        launch_copy_many(cl, s->st);
        break;
      }
      if (relpic_status e = c.advance_e(n)) return e;
      c.swap_b();
    }
    // reverse sweep over n = c1 .. c0 + 1
    for (long long n = c1; n > c0; --n) {
      const long long k = n - c0;
      Real *en[3] = {segE(k, 0), segE(k, 1), segE(k, 2)};
      Real *bn_[3] = {segB(k, 0), segB(k, 1), segB(k, 2)};
      const Real *bn1_3 = segB(k + 1, 2);
      const LossBox lb = c.loss_box(n);
      launch_adj_loss_grad<Real>(c.g, en[0], en[1], bn_[2], bn1_3, lb, c.w, 0.0, 0.5, aE[0], aE[1], aB[2], s->st);
      launch_adj_grad_curl<Real>(c.g, 0, M, aB[1], aB[2], en[1], en[2], c.dt / s->dx[0], dC, s->st);
      launch_adj_loss_grad<Real>(c.g, en[0], en[1], bn_[2], bn1_3, lb, c.w, 1.0, 0.0, aE[0], aE[1], aB[2], s->st);
      c.curl_minus(aE, aB, -c.dt);
      launch_adj_grad_curl<Real>(c.g, 1, M, aE[1], aE[2], bn_[1], bn_[2], c.dt / s->dx[0], dC, s->st);
      if (M > 1)
        launch_adj_grad_jcorr<Real>(c.g, M, aE[0], (const Real *)slot_ptr(a->segJ, c.fb, k - 1),
                                    (const Real *)s->taps, s->ng, a->segbox + (k - 1), c.dt, dC, s->st);
      c.curl_plus(aE, aB, aB, -c.dt);
      launch_adj_loss_grad<Real>(c.g, en[0], en[1], bn_[2], bn1_3, lb, c.w, 0.0, 0.5, aE[0], aE[1], aB[2], s->st);
    }
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(dLdC, dC, sizeof(double) * M, hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  return RELPIC_OK;
}

}  // namespace

extern "C" {

relpic_status relpic_adj_create(const relpic_grid *grid, int M, const double *C0, relpic_precision prec,
                                const relpic_device *dev, int64_t nsteps, int checkpoint_every,
                                const relpic_loss_box *box, relpic_adj **out) {
  return guarded("adj_create", [&]() -> relpic_status {
    if (!grid || !out || !box || !C0) return fail(RELPIC_EINVAL, "adj_create: null argument");
    *out = nullptr;
    if (grid->ndim != 2 || grid->bc1 != RELPIC_BC_PERIODIC)
      return fail(RELPIC_EINVAL, "adj_create: the adjoint runs on a 2D periodic grid");
    if (M < 1 || M > 8) return fail(RELPIC_EINVAL, "adj_create: M must be in 1..8");
    if (nsteps < 1 || nsteps > (1 << 24) || checkpoint_every < 1 || checkpoint_every > 100000)
      return fail(RELPIC_EINVAL, "adj_create: bad step count or checkpoint interval");
    if (!(box->half1 > 0.0) || !(box->half2 > 0.0) || !std::isfinite(box->x1) || !std::isfinite(box->x2) ||
        !std::isfinite(box->v1))
      return fail(RELPIC_EINVAL, "adj_create: bad loss box");
    relpic_solver sol{M, C0};
    relpic_sim *s = nullptr;
    if (relpic_status e = relpic_create(grid, &sol, prec, dev, &s)) return e;
    relpic_adj *a = new (std::nothrow) relpic_adj();
    if (!a) {
      relpic_destroy(s);
      return fail(RELPIC_ENOMEM, "adj_create: host allocation failed");
    }
    a->s = s;
    a->nsteps = nsteps;
    a->every = checkpoint_every;
    a->box = *box;
    a->M = M;
    const size_t fb = s->esz * (size_t)s->N;
    const long long nck = (nsteps + checkpoint_every - 1) / checkpoint_every;
    const long long S = std::min<long long>(checkpoint_every, nsteps);
    a->ckF = dev_alloc(s, fb * 6 * (size_t)nck);
    a->segF = dev_alloc(s, fb * 6 * (size_t)(S + 2));
    a->segJ = M > 1 ? dev_alloc(s, fb * (size_t)S) : nullptr;
    a->segbox = (JBox *)dev_alloc(s, sizeof(JBox) * (size_t)S);
    a->dacc = (double *)dev_alloc(s, sizeof(double) * (1 + kMaxM));
    bool ok = a->ckF && a->segF && (M == 1 || a->segJ) && a->segbox && a->dacc;
    for (int d = 0; d < 3 && ok; ++d) {
      a->aE[d] = dev_alloc(s, fb);
      a->aB[d] = dev_alloc(s, fb);
      ok = a->aE[d] && a->aB[d];
    }
    if (!ok) {
      relpic_destroy(s);
      delete a;
      return fail(RELPIC_ENOMEM, "adj_create: allocation failed");
    }
    *out = a;
    return RELPIC_OK;
  });
}

relpic_status relpic_adj_destroy(relpic_adj *a) {
  return guarded("adj_destroy", [&]() -> relpic_status {
    if (!a) return RELPIC_OK;
    relpic_destroy(a->s);
    delete a;
    return RELPIC_OK;
  });
}

relpic_status relpic_adj_load_particles(relpic_adj *a, double Q, int64_t n, const int32_t *cell, const double *offset,
                                        const double *u) {
  return guarded("adj_load_particles", [&]() -> relpic_status {
    if (relpic_status e = check_adj(a)) return e;
    if (a->nparts > 0 || !a->s->sp.empty()) return fail(RELPIC_ESTATE, "adj_load_particles: particles already loaded");
    if (n < 1 || n >= (1LL << 31)) return fail(RELPIC_EINVAL, "adj_load_particles: bad count");
    relpic_sim *s = a->s;
    int sid = -1;
    if (relpic_status e = relpic_add_species(s, 0.0, Q, n, &sid)) return e;
    if (relpic_status e = relpic_load_particles(s, sid, n, cell, offset, u)) return e;
    if (relpic_status e = relpic_sort_particles(s)) return e;
    a->nparts = (int)s->sp[0].n;
    const long long nck = (a->nsteps + a->every - 1) / a->every;
    // initial state and per-checkpoint copies (each array sized for 8-byte elements)
    const size_t pb = 8 * (size_t)a->nparts;
    for (int k = 0; k < 6; ++k) {
      a->p0[k] = dev_alloc(s, pb);
      if (!a->p0[k]) return fail(RELPIC_ENOMEM, "adj_load_particles: allocation failed");
    }
    a->ckP = dev_alloc(s, pb * 6 * (size_t)nck);
    if (!a->ckP) return fail(RELPIC_ENOMEM, "adj_load_particles: allocation failed");
    if (relpic_status e = particles_copy(a, a->p0, 0)) return e;
    HIP_OK(hipStreamSynchronize(s->st));
    return RELPIC_OK;
  });
}

relpic_status relpic_adj_forward(relpic_adj *a, const double *C, double *loss) {
  return guarded("adj_forward", [&]() -> relpic_status {
    if (relpic_status e = check_adj(a)) return e;
    if (!C || !loss) return fail(RELPIC_EINVAL, "adj_forward: null argument");
    if (a->s->prec == RELPIC_FP32) return do_forward<float>(a, C, loss);
    return do_forward<double>(a, C, loss);
  });
}

relpic_status relpic_adj_backward(relpic_adj *a, double *dLdC) {
  return guarded("adj_backward", [&]() -> relpic_status {
    if (relpic_status e = check_adj(a)) return e;
    if (!dLdC) return fail(RELPIC_EINVAL, "adj_backward: null argument");
    if (!a->forward_done) return fail(RELPIC_ESTATE, "adj_backward: no forward pass with these coefficients");
    if (a->s->prec == RELPIC_FP32) return do_backward<float>(a, dLdC);
    return do_backward<double>(a, dLdC);
  });
}

relpic_status relpic_adj_sim(relpic_adj *a, relpic_sim **sim) {
  return guarded("adj_sim", [&]() -> relpic_status {
    if (relpic_status e = check_adj(a)) return e;
    if (!sim) return fail(RELPIC_EINVAL, "adj_sim: null argument");
    *sim = a->s;
    return RELPIC_OK;
  });
}

}  // extern "C"
