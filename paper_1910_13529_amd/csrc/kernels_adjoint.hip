// Kernels of the adjoint (reverse-mode) field advance on a 2D periodic grid:
// the loss on the fields around a moving bunch, its gradient with respect to
// E and B, and the FP64 reductions that give dL/dC_l (the axial coefficients
// enter both curl operators and the J1 correction G = K^-1 of Sec. 3).
//
// Loss at step n (E^n; B^n = (B^{n-1/2} + B^{n+1/2}) / 2):
//   l_n = w * sum over points outside the bunch box of
//         E1^2 (at E1's point)  +  (E2 - B3c)^2 (at E2's point),
// with B3c the two-point x1 average of B^n_3 onto E2's point (i1, i2 + 1/2).
// The reverse-mode steps reuse the forward curl kernels: the transposes of
// the discrete operators satisfy (curl+)^T = curl-, so the adjoint state
// advances with the forward update and a negated time step.
#include "adjoint_kernels.h"
#include "relpic_internal.h"

namespace relpic {

namespace {

// Whether the point ((i1 + o1) dx1, (i2 + o2) dx2) lies outside the box.
// Rounded products and differences (no fused multiply-add), so that a point
// on the box's edge falls on the same side as in plain double arithmetic.
__device__ __forceinline__ bool outside(const LossBox &b, int i1, double o1, int i2, double o2) {
  const double x1 = __dmul_rn(i1 + o1, b.dx1), x2 = __dmul_rn(i2 + o2, b.dx2);
  return fabs(__dsub_rn(x1, b.c1)) > b.h1 || fabs(__dsub_rn(x2, b.c2)) > b.h2;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// FP64 sum over a workgroup of 256 threads, atomically added to *out
__device__ __forceinline__ void block_add(double v, double *out) {
  __shared__ double part[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

// E2 - B3c at E2's point of cell (i1, i2), in FP64 (B3 given as the two
// half-step buffers a, b)
template <typename Real>
__device__ __forceinline__ double e2_minus_b3(const Geo &g, const Real *E2, const Real *B3a, const Real *B3b, int i1,
                                              long long row) {
  const int im = wrapi(i1 - 1, g.n1);
  const double b3 = 0.25 * ((double)B3a[row + im] + (double)B3b[row + im] + (double)B3a[row + i1] +
                            (double)B3b[row + i1]);
  return (double)E2[row + i1] - b3;
}

template <typename Real>
__global__ __launch_bounds__(256) void k_adj_loss(Geo g, const Real *E1, const Real *E2, const Real *B3a,
                                                  const Real *B3b, LossBox lb, double w, double *out) {
  double acc = 0.0;
  // rows per workgroup, cells per thread (no 64-bit index division)
  for (int i2 = blockIdx.x; i2 < g.n2; i2 += gridDim.x) {
    const long long row = (long long)g.n1 * i2;
    for (int i1 = threadIdx.x; i1 < g.n1; i1 += blockDim.x) {
      if (outside(lb, i1, 0.5, i2, 0.0)) {
        const double e1 = (double)E1[row + i1];
        acc += e1 * e1;
      }
      if (outside(lb, i1, 0.0, i2, 0.5)) {
        const double r = e2_minus_b3(g, E2, B3a, B3b, i1, row);
        acc += r * r;
      }
    }
  }
  block_add(w * acc, out);
}

// aE1 += fe dl/dE1, aE2 += fe dl/dE2, aB3 += fb dl/dB^n_3.  B3c(i1) averages
// B^n_3 at i1 - 1 and i1, so dl/dB^n_3(k) = -w (m r)(k) - w (m r)(k + 1), with
// r = E2 - B3c and m the outside-the-box mask at E2's points.
template <typename Real>
__global__ __launch_bounds__(256) void k_adj_loss_grad(Geo g, const Real *E1, const Real *E2, const Real *B3a,
                                                       const Real *B3b, LossBox lb, double w, double fe, double fb,
                                                       Real *aE1, Real *aE2, Real *aB3) {
  const long long N = (long long)g.n1 * g.n2;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < N; id += (long long)gridDim.x * blockDim.x) {
    const int i1 = (int)(id % g.n1), i2 = (int)(id / g.n1);
    const long long row = id - i1;
    const bool m0 = outside(lb, i1, 0.0, i2, 0.5);
    const double r0 = m0 ? e2_minus_b3(g, E2, B3a, B3b, i1, row) : 0.0;
    if (fe != 0.0) {
      if (outside(lb, i1, 0.5, i2, 0.0)) aE1[id] += (Real)(fe * 2.0 * w * (double)E1[id]);
      if (m0) aE2[id] += (Real)(fe * 2.0 * w * r0);
    }
    if (fb != 0.0) {
      const int ip = wrapi(i1 + 1, g.n1);
      const bool m1 = outside(lb, ip, 0.0, i2, 0.5);
      const double r1 = m1 ? e2_minus_b3(g, E2, B3a, B3b, ip, row) : 0.0;
      aB3[id] += (Real)(fb * (-w) * (r0 + r1));
    }
  }
}

// blockIdx.y = l - 1.  part 0 (T1): sum  bA2 (E3(i+l) - E3(i-l+1)) - bA3 (E2(i+l) - E2(i-l+1))
//                      part 1 (T2): sum -eA2 (B3(i+l-1) - B3(i-l)) + eA3 (B2(i+l-1) - B2(i-l))
// times `scale`, added to out[l - 1].
template <typename Real>
__global__ __launch_bounds__(256) void k_adj_grad_curl_flat(Geo g, int part, const Real *A2, const Real *A3,
                                                       const Real *F2, const Real *F3, double scale, double *out) {
  const int l = blockIdx.y + 1;
  double acc = 0.0;
  const long long N = (long long)g.n1 * g.n2;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < N; id += (long long)gridDim.x * blockDim.x) {
    const int i1 = (int)(id % g.n1);
    const long long row = id - i1;
    if (part == 0) {
      const int p = wrapi(i1 + l, g.n1), m = wrapi(i1 - l + 1, g.n1);
      acc += (double)A2[id] * ((double)F3[row + p] - (double)F3[row + m]) -
             (double)A3[id] * ((double)F2[row + p] - (double)F2[row + m]);
    } else {
      const int p = wrapi(i1 + l - 1, g.n1), m = wrapi(i1 - l, g.n1);
      acc += -(double)A2[id] * ((double)F3[row + p] - (double)F3[row + m]) +
             (double)A3[id] * ((double)F2[row + p] - (double)F2[row + m]);
    }
  }
  block_add(scale * acc, out + (l - 1));
}

// blockIdx.y = l - 1.  T3_l = scale * sum_i J1c(i) sum_{|k| < l} (G aE1)(i + k)
// over the support of J1c (its deposit box widened along x1 by ng), with
// (G v)(j) = sum_{|m| <= ng} g_|m| v(j - m).
template <typename Real>
__global__ __launch_bounds__(256) void k_adj_grad_jcorr(Geo g, const Real *aE1, const Real *J1c, const Real *taps,
                                                        int ng, const JBox *box, double scale, double *out) {
  const int l = blockIdx.y + 1;
  const JBox b = *box;
  double acc = 0.0;
  if (b.hi[0] >= b.lo[0]) {
    int lo1 = b.lo[0] - ng, hi1 = b.hi[0] + ng;
    if (hi1 - lo1 + 1 >= g.n1) {
      lo1 = 0;
      hi1 = g.n1 - 1;
    }
    const long long w1 = hi1 - lo1 + 1, w2 = b.hi[1] - b.lo[1] + 1;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < w1 * w2;
         t += (long long)gridDim.x * blockDim.x) {
      const int i1 = wrapi(lo1 + (int)(t % w1), g.n1);
      const int i2 = b.lo[1] + (int)(t / w1);
      const long long row = (long long)g.n1 * i2;
      const double j = (double)J1c[row + i1];
      if (j == 0.0) continue;
      double s = 0.0;
      for (int k = -(l - 1); k <= l - 1; ++k) {
        const int c = i1 + k;
        double ge = (double)taps[0] * (double)aE1[row + wrapi(c, g.n1)];
        for (int m = 1; m <= ng; ++m)
          ge += (double)taps[m] * ((double)aE1[row + wrapi(c - m, g.n1)] + (double)aE1[row + wrapi(c + m, g.n1)]);
        s += ge;
      }
      acc += j * s;
    }
  }
  block_add(scale * acc, out + (l - 1));
}

// The same sums for every l <= M in one pass (M <= MM): a workgroup takes
// rows of the support, stages the row's aE1 (reach ng + MM - 1 on each side)
// in LDS, forms G aE1 there once, and adds the running sums
// s_l = s_{l-1} + (G aE1)(i - l + 1) + (G aE1)(i + l - 1) per cell.
template <typename Real, int MM>
__global__ __launch_bounds__(256) void k_adj_grad_jcorr_rows(Geo g, int M, const Real *aE1, const Real *J1c,
                                                             const Real *taps, int ng, const JBox *box, double scale,
                                                             double *out) {
  extern __shared__ __align__(16) unsigned char gj_lds[];
  __shared__ double wsum[4][MM];
  const JBox b = *box;
  double acc[MM];
#pragma unroll
  for (int l = 0; l < MM; ++l) acc[l] = 0.0;
  int w2 = 0;
  if (b.hi[0] >= b.lo[0]) {
    int lo1 = b.lo[0] - ng, hi1 = b.hi[0] + ng;
    if (hi1 - lo1 + 1 >= g.n1) {
      lo1 = 0;
      hi1 = g.n1 - 1;
    }
    const int w1 = hi1 - lo1 + 1, h = MM - 1;
    const int na = w1 + 2 * (h + ng), nge = w1 + 2 * h;
    double *ae = reinterpret_cast<double *>(gj_lds);
    double *ge = ae + na;
    w2 = b.hi[1] - b.lo[1] + 1;
    for (int r = blockIdx.x; r < w2; r += gridDim.x) {
      const long long row = (long long)g.n1 * (b.lo[1] + r);
      __syncthreads();  // the previous row's readers are done
      for (int t = threadIdx.x; t < na; t += blockDim.x) ae[t] = (double)aE1[row + wrapi(lo1 - h - ng + t, g.n1)];
      __syncthreads();
      for (int t = threadIdx.x; t < nge; t += blockDim.x) {
        const double *c = ae + ng + t;
        double v = (double)taps[0] * c[0];
        for (int m = 1; m <= ng; ++m) v += (double)taps[m] * (c[-m] + c[m]);
        ge[t] = v;
      }
      __syncthreads();
      for (int t = threadIdx.x; t < w1; t += blockDim.x) {
        const double j = (double)J1c[row + wrapi(lo1 + t, g.n1)];
        if (j == 0.0) continue;
        const double *c = ge + h + t;
        double sl = c[0];
        acc[0] += j * sl;
#pragma unroll
        for (int l = 2; l <= MM; ++l) {
          if (l > M) break;
          sl += c[-(l - 1)] + c[l - 1];
          acc[l - 1] += j * sl;
        }
      }
    }
  }
  if ((int)blockIdx.x >= w2) return;  // no rows here (uniform over the workgroup)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l < MM; ++l) {
    double v = acc[l];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) wsum[wave][l] = v;
  }
  __syncthreads();
  if (threadIdx.x < M) {
    const int l = threadIdx.x;
    atomicAdd(out + l, scale * (wsum[0][l] + wsum[1][l] + wsum[2][l] + wsum[3][l]));
  }
}

// The same sums for every l <= M in one pass (M <= MM): a workgroup takes
// whole x1 rows, stages F2, F3 of a row with MM cells of periodic halo on
// each side in LDS (FP64), and each thread keeps one partial sum per l.
template <typename Real, int MM>
__global__ __launch_bounds__(256) void k_adj_grad_curl_rows(Geo g, int part, int M, const Real *A2, const Real *A3,
                                                            const Real *F2, const Real *F3, double scale,
                                                            double *out) {
  extern __shared__ __align__(16) unsigned char gc_lds[];
  __shared__ double wsum[4][MM];
  const int pitch = g.n1 + 2 * MM;
  double *f2 = reinterpret_cast<double *>(gc_lds);
  double *f3 = f2 + pitch;
  double acc[MM];
#pragma unroll
  for (int l = 0; l < MM; ++l) acc[l] = 0.0;
  for (int r = blockIdx.x; r < g.n2; r += gridDim.x) {
    const long long row = (long long)g.n1 * r;
    __syncthreads();  // the previous row's readers are done
    for (int t = threadIdx.x; t < pitch; t += blockDim.x) {
      const int i = wrapi(t - MM, g.n1);
      f2[t] = (double)F2[row + i];
      f3[t] = (double)F3[row + i];
    }
    __syncthreads();
    for (int i1 = threadIdx.x; i1 < g.n1; i1 += blockDim.x) {
      const double a2 = (double)A2[row + i1], a3 = (double)A3[row + i1];
      const double *c2 = f2 + MM + i1, *c3 = f3 + MM + i1;
#pragma unroll
      for (int l = 1; l <= MM; ++l) {
        if (l > M) break;
        if (part == 0)
          acc[l - 1] += a2 * (c3[l] - c3[1 - l]) - a3 * (c2[l] - c2[1 - l]);
        else
          acc[l - 1] += -a2 * (c3[l - 1] - c3[-l]) + a3 * (c2[l - 1] - c2[-l]);
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l < MM; ++l) {
    double v = acc[l];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) wsum[wave][l] = v;
  }
  __syncthreads();
  if (threadIdx.x < M) {
    const int l = threadIdx.x;
    atomicAdd(out + l, scale * (wsum[0][l] + wsum[1][l] + wsum[2][l] + wsum[3][l]));
  }
}

constexpr int kAdjGrid = 1024;
// the loss sums into one FP64 word: one atomic per workgroup, and
// same-address atomics serialize (1024 of them took ~12 us)
constexpr int kAdjLossBlocks = 128;
constexpr int kGradCurlRowsBlocks = 256;

}  // namespace

template <typename Real>
void launch_adj_loss(const Geo &g, const Real *E1, const Real *E2, const Real *B3a, const Real *B3b,
                     const LossBox &lb, double w, double *out, hipStream_t st) {
  k_adj_loss<Real><<<kAdjLossBlocks, 256, 0, st>>>(g, E1, E2, B3a, B3b, lb, w, out);
}

template <typename Real>
void launch_adj_loss_grad(const Geo &g, const Real *E1, const Real *E2, const Real *B3a, const Real *B3b,
                          const LossBox &lb, double w, double fe, double fb, Real *aE1, Real *aE2, Real *aB3,
                          hipStream_t st) {
  k_adj_loss_grad<Real><<<kAdjGrid, 256, 0, st>>>(g, E1, E2, B3a, B3b, lb, w, fe, fb, aE1, aE2, aB3);
}

template <typename Real>
void launch_adj_grad_curl(const Geo &g, int part, int M, const Real *A2, const Real *A3, const Real *F2, const Real *F3,
                          double scale, double *out, hipStream_t st) {
  const int MM = M <= 4 ? 4 : (M <= 8 ? 8 : (M <= 16 ? 16 : kMaxM));
  const size_t lds = 2 * sizeof(double) * (size_t)(g.n1 + 2 * MM);
  if (M > kMaxM || lds > 49152) {
    k_adj_grad_curl_flat<Real><<<dim3(kAdjGrid / 4, M), 256, 0, st>>>(g, part, A2, A3, F2, F3, scale, out);
    return;
  }
  const unsigned blocks = (unsigned)(g.n2 < kGradCurlRowsBlocks ? g.n2 : kGradCurlRowsBlocks);
  if (MM == 4)
    k_adj_grad_curl_rows<Real, 4><<<blocks, 256, lds, st>>>(g, part, M, A2, A3, F2, F3, scale, out);
  else if (MM == 8)
    k_adj_grad_curl_rows<Real, 8><<<blocks, 256, lds, st>>>(g, part, M, A2, A3, F2, F3, scale, out);
  else if (MM == 16)
    k_adj_grad_curl_rows<Real, 16><<<blocks, 256, lds, st>>>(g, part, M, A2, A3, F2, F3, scale, out);
  else
    k_adj_grad_curl_rows<Real, kMaxM><<<blocks, 256, lds, st>>>(g, part, M, A2, A3, F2, F3, scale, out);
}

template <typename Real>
void launch_adj_grad_jcorr(const Geo &g, int M, const Real *aE1, const Real *J1c, const Real *taps, int ng,
                           const JBox *box, double scale, double *out, hipStream_t st) {
  const int MM = M <= 4 ? 4 : (M <= 8 ? 8 : (M <= 16 ? 16 : kMaxM));
  const size_t lds = sizeof(double) * (size_t)(2 * g.n1 + 4 * (MM - 1) + 2 * ng);
  if (M > kMaxM || lds > 49152) {
    k_adj_grad_jcorr<Real><<<dim3(64, M), 256, 0, st>>>(g, aE1, J1c, taps, ng, box, scale, out);
    return;
  }
  if (MM == 4)
    k_adj_grad_jcorr_rows<Real, 4><<<64, 256, lds, st>>>(g, M, aE1, J1c, taps, ng, box, scale, out);
  else if (MM == 8)
    k_adj_grad_jcorr_rows<Real, 8><<<64, 256, lds, st>>>(g, M, aE1, J1c, taps, ng, box, scale, out);
  else if (MM == 16)
    k_adj_grad_jcorr_rows<Real, 16><<<64, 256, lds, st>>>(g, M, aE1, J1c, taps, ng, box, scale, out);
  else
    k_adj_grad_jcorr_rows<Real, kMaxM><<<64, 256, lds, st>>>(g, M, aE1, J1c, taps, ng, box, scale, out);
}

// Grid-stride copy of every op: 16-byte words where both pointers and the
// size allow it, else 4-byte words, else bytes.
__global__ __launch_bounds__(256) void k_copy_many(CopyList list) {
  const size_t t0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
  for (int k = 0; k < list.n; ++k) {
    const CopyOp o = list.op[k];
    const uintptr_t al = (uintptr_t)o.dst | (uintptr_t)o.src | (uintptr_t)o.bytes;
    if ((al & 15) == 0) {
      uint4 *d = (uint4 *)o.dst;
      const uint4 *sr = (const uint4 *)o.src;
      for (size_t i = t0; i < o.bytes / 16; i += stride) d[i] = sr[i];
    } else if ((al & 3) == 0) {
      unsigned *d = (unsigned *)o.dst;
      const unsigned *sr = (const unsigned *)o.src;
      for (size_t i = t0; i < o.bytes / 4; i += stride) d[i] = sr[i];
    } else {
      unsigned char *d = (unsigned char *)o.dst;
      const unsigned char *sr = (const unsigned char *)o.src;
      for (size_t i = t0; i < o.bytes; i += stride) d[i] = sr[i];
    }
  }
}

void launch_copy_many(const CopyList &list, hipStream_t st) {
  if (list.n <= 0) return;
  size_t words = 0;
  for (int k = 0; k < list.n; ++k) words = list.op[k].bytes / 16 > words ? list.op[k].bytes / 16 : words;
  const size_t want = (words + 255) / 256;
  k_copy_many<<<(unsigned)(want < 1 ? 1 : (want > 2048 ? 2048 : want)), 256, 0, st>>>(list);
}

#define RELPIC_INST_ADJ(Real)                                                                                      \
  template void launch_adj_loss<Real>(const Geo &, const Real *, const Real *, const Real *, const Real *,         \
                                      const LossBox &, double, double *, hipStream_t);                            \
  template void launch_adj_loss_grad<Real>(const Geo &, const Real *, const Real *, const Real *, const Real *,    \
                                           const LossBox &, double, double, double, Real *, Real *, Real *,       \
                                           hipStream_t);                                                          \
  template void launch_adj_grad_curl<Real>(const Geo &, int, int, const Real *, const Real *, const Real *,        \
                                           const Real *, double, double *, hipStream_t);                           \
  template void launch_adj_grad_jcorr<Real>(const Geo &, int, const Real *, const Real *, const Real *, int,       \
                                            const JBox *, double, double *, hipStream_t);

RELPIC_INST_ADJ(float)
RELPIC_INST_ADJ(double)

}  // namespace relpic
