// FP64 diagnostics (energies, charge, discrete Gauss residual) and plasma
// injection for the moving window.  Diagnostics accumulate in FP64 whatever
// the field precision, so FP32 runs report energy and charge conservation at
// FP64 resolution.
#include <climits>

#include "kernels.h"

namespace relpic {

constexpr int kRedBlock = 256;

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[kRedBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;  // valid in thread 0
}

__device__ __forceinline__ double block_max(double v) {
  __shared__ double sh[kRedBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = fmax(t, sh[w]);
  return t;
}

// non-negative doubles order like their bit patterns
__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

template <typename Real>
__global__ __launch_bounds__(kRedBlock) void k_field_energy(Geo g, Fields<Real> f, double *acc) {
  double s = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N; i += (long long)gridDim.x * blockDim.x) {
    const double e1 = f.E1[i], e2 = f.E2[i], e3 = f.E3[i], b1 = f.B1[i], b2 = f.B2[i], b3 = f.B3[i];
    s += e1 * e1 + e2 * e2 + e3 * e3 + b1 * b1 + b2 * b2 + b3 * b3;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) atomicAdd(acc, 0.5 * s);
}

template <typename Real>
__global__ __launch_bounds__(kRedBlock) void k_kinetic(Particles<Real> p, double mass, double *acc,
                                                       unsigned long long *cnt) {
  double s = 0;
  double c = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p.n; i += (long long)gridDim.x * blockDim.x) {
    if (p.cell[i] < 0) continue;
    const double u1 = p.u1[i], u2 = p.u2[i], u3 = p.u3[i];
    const double usq = u1 * u1 + u2 * u2 + u3 * u3;
    // gamma - 1 without cancellation
    s += mass * usq / (sqrt(1.0 + usq) + 1.0);
    c += 1.0;
  }
  s = block_sum(s);
  __syncthreads();
  c = block_sum(c);
  if (threadIdx.x == 0) {
    atomicAdd(acc, s);
    atomicAdd(cnt, (unsigned long long)c);
  }
}

// rho of the particles (FP64).  A workgroup takes kRhoChunk consecutive
// particles and finds the bounding box of their cells.  When that box, grown
// by the one-node reach of the quadratic shape on each side, fits kRhoTile
// doubles of LDS (always for cell-sorted particles of a bunch), every particle
// adds its 3 x 3 (x 3) node weights to the LDS tile, and the tile is added to
// rho with one atomic per non-zero node; hot nodes of a dense bunch then see
// one global atomic per workgroup instead of one per particle.  Otherwise
// (scattered or unsorted particles) each weight goes to rho directly.
constexpr int kRhoChunk = 2048;
constexpr int kRhoTile = 6144;

template <typename Real, int DIM>
__device__ __forceinline__ bool rho_cell(const Geo &g, const Particles<Real> &p, long long i, int c[3]) {
  const int packed = p.cell[i];
  if (packed < 0) return false;
  int s1;
  unpack_cell(g, packed, s1, c[1], c[2]);
  c[0] = s1 - g.ws_mod;  // window-relative x1 cell
  if (c[0] < 0) c[0] += g.n1;
  return true;
}

template <typename Real, int DIM>
__global__ __launch_bounds__(kRedBlock) void k_rho(Geo g, Particles<Real> p, double qdv, double *rho) {
  __shared__ double tile[kRhoTile];
  __shared__ int wlo[3][kRedBlock / 64], whi[3][kRedBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long base = blockIdx.x * (long long)kRhoChunk;
  const long long end = base + kRhoChunk < p.n ? base + kRhoChunk : p.n;
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  for (long long i = base + threadIdx.x; i < end; i += kRedBlock) {
    int c[3];
    if (!rho_cell<Real, DIM>(g, p, i, c)) continue;
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], c[d]);
      hi[d] = max(hi[d], c[d]);
    }
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
      hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
    }
  if (lane == 0)
    for (int d = 0; d < 3; ++d) {
      wlo[d][wave] = lo[d];
      whi[d][wave] = hi[d];
    }
  __syncthreads();
  for (int d = 0; d < 3; ++d)
    for (int w = 0; w < kRedBlock / 64; ++w) {
      lo[d] = min(lo[d], wlo[d][w]);
      hi[d] = max(hi[d], whi[d][w]);
    }
  if (lo[0] == INT_MAX) return;  // no live particle in the chunk (uniform over the workgroup)
  // tile index (a, b, c) <-> node (lo1 - 1 + a, lo2 - 1 + b, lo3 - 1 + c)
  const int w1 = hi[0] - lo[0] + 3, w2 = hi[1] - lo[1] + 3;
  const long long vol = (long long)w1 * w2 * (DIM == 3 ? hi[2] - lo[2] + 3 : 1);
  const bool fits = vol <= kRhoTile;
  if (fits)
    for (int t = threadIdx.x; t < vol; t += kRedBlock) tile[t] = 0.0;
  __syncthreads();
  for (long long i = base + threadIdx.x; i < end; i += kRedBlock) {
    int c[3];
    if (!rho_cell<Real, DIM>(g, p, i, c)) continue;
    const double o[3] = {(double)p.o1[i], (double)p.o2[i], DIM == 3 ? (double)p.o3[i] : 0.0};
    double w[3][3] = {{0, 0, 0}, {0, 0, 0}, {1, 0, 0}};
    for (int d = 0; d < DIM; ++d) {
      const double a = 0.5 - o[d], b = 0.5 + o[d];
      w[d][0] = 0.5 * a * a;
      w[d][1] = 0.75 - o[d] * o[d];
      w[d][2] = 0.5 * b * b;
    }
    for (int cc = 0; cc < (DIM == 3 ? 3 : 1); ++cc) {
      const double w3 = qdv * w[2][cc];
      for (int bb = 0; bb < 3; ++bb) {
        const double w23 = w3 * w[1][bb];
        if (fits) {
          const int t0 = ((DIM == 3 ? c[2] - lo[2] + cc : 0) * w2 + c[1] - lo[1] + bb) * w1 + c[0] - lo[0];
          for (int aa = 0; aa < 3; ++aa) atomicAdd(&tile[t0 + aa], w23 * w[0][aa]);
        } else {
          const int i3 = DIM == 3 ? wrap(c[2] - 1 + cc, g.n3) : 0;
          const long long row = (long long)g.n1 * (wrap(c[1] - 1 + bb, g.n2) + (long long)g.n2 * i3);
          for (int aa = 0; aa < 3; ++aa) {
            const int col = col_of(g, c[0] - 1 + aa);
            if (col >= 0) atomicAdd(rho + row + col, w23 * w[0][aa]);
          }
        }
      }
    }
  }
  if (!fits) return;
  __syncthreads();
  for (int t = threadIdx.x; t < vol; t += kRedBlock) {
    const double v = tile[t];
    if (v == 0.0) continue;
    const int a = t % w1, b = (t / w1) % w2, cz = t / (w1 * w2);
    const int col = col_of(g, lo[0] - 1 + a);
    if (col < 0) continue;
    const int i3 = DIM == 3 ? wrap(lo[2] - 1 + cz, g.n3) : 0;
    atomicAdd(rho + (long long)g.n1 * (wrap(lo[1] - 1 + b, g.n2) + (long long)g.n2 * i3) + col, v);
  }
}

template <typename Real, int DIM>
__global__ __launch_bounds__(kRedBlock) void k_gauss(Geo g, Fields<Real> f, Axial<double> c1dx, double idx2,
                                                     double idx3, const double *rho, const double *rho_bg,
                                                     int margin1, double *out) {
  double rmax = 0, qmax = 0, qsum = 0;
  for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < g.N;
       id += (long long)gridDim.x * blockDim.x) {
    // id enumerates window cells in logical order
    const int l1 = (int)(id % g.n1);
    const long long rest = id / g.n1;
    const int i2 = (int)(rest % g.n2);
    const int i3 = (int)(rest / g.n2);
    const long long row = (long long)g.n1 * (i2 + (long long)g.n2 * i3);
    const int s1 = col_of(g, l1);
    const long long sid = row + s1;
    double div = 0;
    for (int l = 1; l <= c1dx.M; ++l) {
      const int a = col_of(g, l1 + l - 1), b = col_of(g, l1 - l);
      const double fa = a >= 0 ? (double)f.E1[row + a] : 0.0;
      const double fb = b >= 0 ? (double)f.E1[row + b] : 0.0;
      div += c1dx.c[l - 1] * (fa - fb);
    }
    const long long row2m = (long long)g.n1 * (wrap(i2 - 1, g.n2) + (long long)g.n2 * i3);
    div += idx2 * ((double)f.E2[sid] - (double)f.E2[row2m + s1]);
    if (DIM == 3) {
      const long long row3m = (long long)g.n1 * (i2 + (long long)g.n2 * wrap(i3 - 1, g.n3));
      div += idx3 * ((double)f.E3[sid] - (double)f.E3[row3m + s1]);
    }
    double r = rho[sid];
    qsum += r;
    qmax = fmax(qmax, fabs(r));
    if (rho_bg) r += rho_bg[sid];
    if (!g.window || (l1 >= margin1 && l1 < g.n1 - margin1)) rmax = fmax(rmax, fabs(div - r));
  }
  rmax = block_max(rmax);
  __syncthreads();
  qmax = block_max(qmax);
  __syncthreads();
  qsum = block_sum(qsum);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(out + 0, rmax);
    atomic_max_nonneg(out + 1, qmax);
    atomicAdd(out + 2, qsum);
  }
}

// ---- splitmix64 counter stream (Steele, Lea, Flood 2014) ------------------------
__device__ __forceinline__ unsigned long long smix(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double uni53(unsigned long long seed, unsigned long long k) {
  const unsigned long long z = smix(seed + (k + 1ULL) * 0x9e3779b97f4a7c15ULL);
  return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
__device__ __forceinline__ double normal_k(unsigned long long seed, unsigned long long k) {
  const double a = uni53(seed, 2ULL * k), b = uni53(seed, 2ULL * k + 1ULL);
  return sqrt(-2.0 * log(a)) * cospi(2.0 * b);
}

// A slab of ppc1 x ppc2 x ppc3 particles per cell in window cell win_cell.
// Particle r of the slab in row order (cell index i2 + n2 i3, then the
// sub-lattice point) carries id id0 + r and the thermal momenta of counter
// counter0 + r.  2D stores them in that order; 3D stores the cells in
// kInjBlock x kInjBlock transverse blocks (narrower at the x2 and x3 ends;
// x2 blocks fastest, x2 fastest inside a block), so that a push chunk of one
// block's particles covers a 5 x 12 x 12 deposit box, which the push holds
// in LDS, instead of a long x2 row.
template <typename Real>
__global__ void k_inject(int ndim, Geo g, Particles<Real> p, int *id, long long first, int win_cell, int ppc1,
                         int ppc2, int ppc3, double uth, unsigned long long seed, unsigned long long counter0,
                         long long id0) {
  const long long per = (long long)ppc1 * ppc2 * ppc3;
  const long long total = per * g.n2 * g.n3;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= total) return;
  const long long q = t % per;
  const long long rc = t / per;  // the cell's place in storage order
  int i2, i3;
  if (ndim == 3) {
    // block row b3 (h3 rows of cells), then block b2 (w2 x h3 cells) in it
    const long long rowcells = (long long)kInjBlock * g.n2;
    const int b3 = (int)(rc / rowcells);
    const int h3 = min(kInjBlock, g.n3 - kInjBlock * b3);
    const long long rr = rc - (long long)b3 * rowcells;
    const int b2 = (int)(rr / (kInjBlock * h3));
    const int w2 = min(kInjBlock, g.n2 - kInjBlock * b2);
    const int sb = (int)(rr - (long long)b2 * kInjBlock * h3);
    i2 = kInjBlock * b2 + sb % w2;
    i3 = kInjBlock * b3 + sb / w2;
  } else {
    i2 = (int)(rc % g.n2);
    i3 = (int)(rc / g.n2);
  }
  const long long r = ((long long)i3 * g.n2 + i2) * per + q;  // row-order index
  const int a = (int)(q % ppc1), b = (int)((q / ppc1) % ppc2), c = (int)(q / ((long long)ppc1 * ppc2));
  const long long k = first + t;
  const int s1 = col_of(g, win_cell);
  p.cell[k] = s1 + g.n1 * (i2 + g.n2 * i3);
  id[k] = (int)(id0 + r);
  p.o1[k] = (Real)((a + 0.5) / ppc1 - 0.5);
  p.o2[k] = (Real)((b + 0.5) / ppc2 - 0.5);
  if (ndim == 3) p.o3[k] = (Real)((c + 0.5) / ppc3 - 0.5);
  const unsigned long long ctr = counter0 + (unsigned long long)r;
  p.u1[k] = (Real)(uth * normal_k(seed, 3ULL * ctr + 0ULL));
  p.u2[k] = (Real)(uth * normal_k(seed, 3ULL * ctr + 1ULL));
  p.u3[k] = (Real)(uth * normal_k(seed, 3ULL * ctr + 2ULL));
}

// ---- launchers --------------------------------------------------------------------

static unsigned red_blocks(long long n) {
  long long b = (n + kRedBlock - 1) / kRedBlock;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <typename Real>
void launch_diag_field_energy(const Geo &g, const Fields<Real> &f, double *acc, hipStream_t st) {
  k_field_energy<Real><<<red_blocks(g.N), kRedBlock, 0, st>>>(g, f, acc);
}

template <typename Real>
void launch_diag_kinetic(const Particles<Real> &p, double mass, double *acc, unsigned long long *cnt,
                         hipStream_t st) {
  if (p.n <= 0) return;
  k_kinetic<Real><<<red_blocks(p.n), kRedBlock, 0, st>>>(p, mass, acc, cnt);
}

template <typename Real>
void launch_diag_rho(int ndim, const Geo &g, const Particles<Real> &p, double qdv, double *rho, hipStream_t st) {
  if (p.n <= 0) return;
  const unsigned blocks = (unsigned)((p.n + kRhoChunk - 1) / kRhoChunk);
  if (ndim == 3)
    k_rho<Real, 3><<<blocks, kRedBlock, 0, st>>>(g, p, qdv, rho);
  else
    k_rho<Real, 2><<<blocks, kRedBlock, 0, st>>>(g, p, qdv, rho);
}

template <typename Real>
void launch_diag_gauss(int ndim, const Geo &g, const Fields<Real> &f, const Axial<double> &c1dx, double idx2,
                       double idx3, const double *rho, const double *rho_bg, int margin1, double *out,
                       hipStream_t st) {
  if (ndim == 3)
    k_gauss<Real, 3><<<red_blocks(g.N), kRedBlock, 0, st>>>(g, f, c1dx, idx2, idx3, rho, rho_bg, margin1, out);
  else
    k_gauss<Real, 2><<<red_blocks(g.N), kRedBlock, 0, st>>>(g, f, c1dx, idx2, idx3, rho, rho_bg, margin1, out);
}

template <typename Real>
void launch_inject_slab(int ndim, const Geo &g, Particles<Real> p, int *id, long long first, int win_cell, int ppc1,
                        int ppc2, int ppc3, double uth, unsigned long long seed, unsigned long long counter0,
                        long long id0, hipStream_t st) {
  const long long total = (long long)ppc1 * ppc2 * ppc3 * g.n2 * g.n3;
  k_inject<Real><<<(unsigned)((total + 255) / 256), 256, 0, st>>>(ndim, g, p, id, first, win_cell, ppc1, ppc2, ppc3,
                                                                    uth, seed, counter0, id0);
}

#define RELPIC_INST_AUX(Real)                                                                                      \
  template void launch_diag_field_energy<Real>(const Geo &, const Fields<Real> &, double *, hipStream_t);          \
  template void launch_diag_kinetic<Real>(const Particles<Real> &, double, double *, unsigned long long *,         \
                                          hipStream_t);                                                            \
  template void launch_diag_rho<Real>(int, const Geo &, const Particles<Real> &, double, double *, hipStream_t);   \
  template void launch_diag_gauss<Real>(int, const Geo &, const Fields<Real> &, const Axial<double> &, double,      \
                                        double, const double *, const double *, int, double *, hipStream_t);       \
  template void launch_inject_slab<Real>(int, const Geo &, Particles<Real>, int *, long long, int, int, int, int,   \
                                         double, unsigned long long, unsigned long long, long long, hipStream_t);

RELPIC_INST_AUX(float)
RELPIC_INST_AUX(double)


// ---- fields at the particles (self-force diagnostic) ------------------------------
// E^n and B^n interpolated at each particle with the push's quadratic
// B-spline, each component from its own staggered points (E1 at (i1+1/2, i2,
// i3), B3 at (i1+1/2, i2+1/2, i3), ...), in FP64.  B is the canonical B^n
// held between relpic_step calls.  out[6 i + c] for particles first .. first
// + count - 1; dropped particles give zeros.

// weights at nodes c-1, c, c+1 (half = 0) or at half points j+1/2 with
// j = the returned start - 1 .. start + 1 (half = 1) for offset o in [-1/2, 1/2)
__device__ __forceinline__ int aux_weights(int c, double o, int half, double w[3]) {
  double d = o;
  int mid = c;
  if (half) {
    if (o >= 0.0) {
      d = o - 0.5;
    } else {
      d = o + 0.5;
      mid = c - 1;
    }
  }
  const double a = 0.5 - d, b = 0.5 + d;
  w[0] = 0.5 * a * a;
  w[1] = 0.75 - d * d;
  w[2] = 0.5 * b * b;
  return mid;
}

template <typename Real, int DIM>
__global__ __launch_bounds__(kRedBlock) void k_gather_at_particles(Geo g, Fields<Real> f, Particles<Real> p,
                                                                    long long first, long long count, double *out) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= count) return;
  const long long i = first + k;
  const int packed = p.cell[i];
  double res[6] = {0, 0, 0, 0, 0, 0};
  if (packed >= 0) {
    int s1, c2, c3;
    unpack_cell(g, packed, s1, c2, c3);
    int c1 = s1 - g.ws_mod;
    if (c1 < 0) c1 += g.n1;
    const int cc[3] = {c1, c2, c3};
    const double o[3] = {(double)p.o1[i], (double)p.o2[i], DIM == 3 ? (double)p.o3[i] : 0.0};
    const Real *F[6] = {f.E1, f.E2, f.E3, f.B1, f.B2, f.B3};
    // half-integer staggering per component and axis
    const int H[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
    for (int c = 0; c < 6; ++c) {
      double w[3][3];
      int mid[3] = {0, 0, 0};
      for (int d = 0; d < 3; ++d) {
        if (d < DIM) {
          mid[d] = aux_weights(cc[d], o[d], H[c][d], w[d]);
        } else {
          w[d][0] = w[d][2] = 0.0;
          w[d][1] = 1.0;
        }
      }
      double acc = 0.0;
      for (int kc = (DIM == 3 ? 0 : 1); kc < (DIM == 3 ? 3 : 2); ++kc) {
        const int i3 = DIM == 3 ? wrap(mid[2] - 1 + kc, g.n3) : 0;
        for (int kb = 0; kb < 3; ++kb) {
          const int i2 = wrap(mid[1] - 1 + kb, g.n2);
          for (int ka = 0; ka < 3; ++ka) {
            const int col = col_of(g, mid[0] - 1 + ka);
            if (col < 0) continue;  // outside the moving window: zero
            const long long id = (long long)g.n1 * (i2 + (long long)g.n2 * i3) + col;
            acc += w[0][ka] * w[1][kb] * w[2][kc] * (double)F[c][id];
          }
        }
      }
      res[c] = acc;
    }
  }
  for (int c = 0; c < 6; ++c) out[6 * k + c] = res[c];
}

template <typename Real>
void launch_gather_at_particles(int ndim, const Geo &g, const Fields<Real> &f, const Particles<Real> &p,
                                long long first, long long count, double *out, hipStream_t st) {
  if (count <= 0) return;
  const unsigned nb = (unsigned)((count + kRedBlock - 1) / kRedBlock);
  if (ndim == 3)
    k_gather_at_particles<Real, 3><<<nb, kRedBlock, 0, st>>>(g, f, p, first, count, out);
  else
    k_gather_at_particles<Real, 2><<<nb, kRedBlock, 0, st>>>(g, f, p, first, count, out);
}
template void launch_gather_at_particles<float>(int, const Geo &, const Fields<float> &, const Particles<float> &,
                                                long long, long long, double *, hipStream_t);
template void launch_gather_at_particles<double>(int, const Geo &, const Fields<double> &, const Particles<double> &,
                                                 long long, long long, double *, hipStream_t);

}  // namespace relpic
