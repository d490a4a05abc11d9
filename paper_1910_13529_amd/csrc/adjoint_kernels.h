// Adjoint kernels of relpic (internal): loss around a moving bunch, its
// gradient with respect to the fields, and the dL/dC_l reductions.  2D,
// periodic grids.
#pragma once

#include "relpic_internal.h"

namespace relpic {

// Excluded box of one step: centre (c1, c2) and half-widths (h1, h2) in
// physical units; dx1, dx2 the cell sizes.
struct LossBox {
  double c1, c2, h1, h2, dx1, dx2;
};

// *out += w * sum outside the box of E1^2 + (E2 - B3c)^2 (FP64)
template <typename Real>
void launch_adj_loss(const Geo &g, const Real *E1, const Real *E2, const Real *B3a, const Real *B3b,
                     const LossBox &lb, double w, double *out, hipStream_t st);
// aE1, aE2 += fe * dl/dE; aB3 += fb * dl/dB^n_3 (B^n = (B3a + B3b) / 2)
template <typename Real>
void launch_adj_loss_grad(const Geo &g, const Real *E1, const Real *E2, const Real *B3a, const Real *B3b,
                          const LossBox &lb, double w, double fe, double fb, Real *aE1, Real *aE2, Real *aB3,
                          hipStream_t st);
// out[l-1] += scale * <A, d(curl)/dC_l F> for l = 1..M; part 0: A = adjoint B,
// F = E (forward operator); part 1: A = adjoint E, F = B (backward operator)
template <typename Real>
void launch_adj_grad_curl(const Geo &g, int part, int M, const Real *A2, const Real *A3, const Real *F2, const Real *F3,
                          double scale, double *out, hipStream_t st);
// out[l-1] += scale * <G S_l J1c, aE1> over J1c's support (box widened by ng)
template <typename Real>
void launch_adj_grad_jcorr(const Geo &g, int M, const Real *aE1, const Real *J1c, const Real *taps, int ng,
                           const JBox *box, double scale, double *out, hipStream_t st);

// Up to kCopyOps device-to-device copies in one launch (the per-step
// segment stores of the reverse pass; separate copies cost a launch each).
constexpr int kCopyOps = 8;
struct CopyOp {
  void *dst;
  const void *src;
  size_t bytes;
};
struct CopyList {
  CopyOp op[kCopyOps];
  int n;
};
void launch_copy_many(const CopyList &list, hipStream_t st);

}  // namespace relpic
