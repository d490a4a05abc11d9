// Particle phase of one PIC step (Sec. 1): quadratic-spline gather of E^n,
// B^n at x^n, relativistic Boris push, cell + offset position update and the
// charge-conserving (Esirkepov) current deposit J^{n+1/2}, fused in one pass
// over the particle arrays so each particle's state is read and written once.
//
// Positions are (packed storage cell, offset in [-1/2, 1/2) cell units), so
// FP32 offsets keep full precision at any distance from the origin.
//
// Deposit.  Particles are kept sorted by cell, so the 64 lanes of a wavefront
// mostly share one or two neighbouring cells of one (x2, x3) row.  Each
// workgroup walks a contiguous chunk of particles, stages E and B over the
// chunk's cells in LDS for the gather, and accumulates current in an LDS tile
// over the same cells; at the end it adds the non-zero tile entries to J in
// HBM with one atomic each.  Inside a wavefront, lanes whose stencils share
// the wavefront's boxes (exact supports when no transverse cell is crossed)
// first sum their contributions with a recursive-halving reduce-scatter over
// the 64 lanes (each lane ends up owning one point per component), so a dense
// bunch costs a few cross-lane moves per particle instead of ~60 conflicting
// atomics.  Other lanes add their stencil to the tile directly.  The device
// code lives in particle_chunk.h, shared with the batched kernels.
#include "particle_chunk.h"

namespace relpic {

// Workgroup b takes sort tile b's particles (b < pc.ntiles) or the b -
// pc.ntiles-th run of 256 K particles after the first pc.nsorted.
template <typename Real, int DIM, int W, bool ROUNDS = true>
__global__ __launch_bounds__(kPushBlock) void k_push_deposit(Geo g, Fields<Real> f, HalfB<Real> Bh,
                                                             Particles<Real> p, PushParams<Real> q, PushChunks pc,
                                                             JBox *blockbox, int *err) {
  constexpr int TILE = PushTile<Real>::bytes;
  __shared__ __align__(16) unsigned char tile_raw[TILE];
  __shared__ int box[kChunkBoxInts];
  const long long b = blockIdx.x;
  long long c0, c1;
  if (b < pc.ntiles) {
    c0 = pc.first[b];
    c1 = pc.end[b];
  } else {
    const long long per = (long long)kPushBlock * pc.K;
    c0 = pc.nsorted + (b - pc.ntiles) * per;
    c1 = c0 + per;
  }
  if constexpr (W == 4) {
    __shared__ GroupLds grp;
    push_chunk<Real, DIM, W, TILE, ROUNDS>(g, f, Bh, p, q, c0, c1, blockbox + b, err, tile_raw, box, &grp);
  } else {
    push_chunk<Real, DIM, W, TILE>(g, f, Bh, p, q, c0, c1, blockbox + b, err, tile_raw, box);
  }
}

// Box of a set of per-workgroup boxes merged into *out: each workgroup
// reduces its share (at least 2048 boxes, at most 256 workgroups) and adds
// one min/max per axis, so the single box sees few atomics.
constexpr int kMergeMaxBlocks = 256;

__global__ __launch_bounds__(256) void k_merge_boxes(const JBox *boxes, long long nbox, JBox *out) {
  __shared__ int wlo[3][4], whi[3][4];
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {-INT_MAX, -INT_MAX, -INT_MAX};
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < nbox; b += (long long)gridDim.x * blockDim.x)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], boxes[b].lo[d]);
      hi[d] = max(hi[d], boxes[b].hi[d]);
    }
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
      hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
    }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      wlo[d][wave] = lo[d];
      whi[d][wave] = hi[d];
    }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int l = min(min(wlo[d][0], wlo[d][1]), min(wlo[d][2], wlo[d][3]));
      const int h = max(max(whi[d][0], whi[d][1]), max(whi[d][2], whi[d][3]));
      if (l <= h) {
        atomicMin(&out->lo[d], l);
        atomicMax(&out->hi[d], h);
      }
    }
}

bool sort_tiles_fit(const Geo &g) {
  const unsigned long long span = (unsigned long long)((g.n1 + 7) / 8 * 8) * (unsigned long long)((g.n2 + 3) / 4 * 4) *
                                  (unsigned long long)(g.n3 > 1 ? (g.n3 + 3) / 4 * 4 : 1);
  return span < 0xFFFFFFFFull;
}

long long push_blocks(long long n, int K) {
  const long long per = (long long)kPushBlock * K;
  return n <= 0 ? 0 : (n + per - 1) / per;
}

long long push_grid(const PushChunks &pc, long long n) {
  return n <= 0 ? 0 : pc.ntiles + push_blocks(n - pc.nsorted, pc.K);
}

template <typename Real>
void launch_push_deposit(int ndim, const Geo &g, const Fields<Real> &f, const HalfB<Real> &Bh,
                         const Particles<Real> &p, const PushParams<Real> &q, const PushChunks &pc, bool wide,
                         bool long_runs, JBox *blockbox, int *err, hipStream_t st) {
  if (p.n <= 0) return;
  const unsigned blocks = (unsigned)push_grid(pc, p.n);
  // FP64 keeps the narrow rounds: the wide ones take it from two waves per SIMD to one
  if (ndim == 3 && wide && long_runs)
    k_push_deposit<Real, 3, 4, false><<<blocks, kPushBlock, 0, st>>>(g, f, Bh, p, q, pc, blockbox, err);
  else if (ndim == 3 && wide && sizeof(Real) == 4)
    k_push_deposit<Real, 3, 4><<<blocks, kPushBlock, 0, st>>>(g, f, Bh, p, q, pc, blockbox, err);
  else if (ndim == 3)
    k_push_deposit<Real, 3, 2><<<blocks, kPushBlock, 0, st>>>(g, f, Bh, p, q, pc, blockbox, err);
  else
    k_push_deposit<Real, 2, 2><<<blocks, kPushBlock, 0, st>>>(g, f, Bh, p, q, pc, blockbox, err);
}

// Particle index range of each sort tile in a tile-sorted array of n alive
// particles: first[t] at the tile's first particle, end[t] one past its last
// (tiles without particles keep the zeros the caller cleared).
__global__ __launch_bounds__(256) void k_tile_ranges(const unsigned *keys, long long n, int shift, long long ntiles,
                                                     int *first, int *end) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const unsigned t = keys[i] >> shift;
  if ((long long)t >= ntiles) return;
  if (i == 0 || (keys[i - 1] >> shift) != t) first[t] = (int)i;
  if (i + 1 == n || (keys[i + 1] >> shift) != t) end[t] = (int)(i + 1);
}

void launch_tile_ranges(const unsigned *keys, long long n, int shift, long long ntiles, int *first, int *end,
                        hipStream_t st) {
  if (n <= 0) return;
  k_tile_ranges<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(keys, n, shift, ntiles, first, end);
}

void launch_merge_boxes(const JBox *blockbox, long long nbox, JBox *jbox, hipStream_t st) {
  if (nbox <= 0) return;
  const long long want = (nbox + 2047) / 2048;
  k_merge_boxes<<<(unsigned)(want < kMergeMaxBlocks ? want : kMergeMaxBlocks), 256, 0, st>>>(blockbox, nbox, jbox);
}

// ---- particle sort (cell order) ---------------------------------------------------

// Counting sort of the particles by cell key (keys below nkeys; dropped
// particles carry 0xFFFFFFFF and are left out): a histogram of the keys, an
// exclusive scan of it (bucket starts, the alive count and the occupied
// cells), and a scatter of each particle index to its bucket.  The array is
// mostly in order already (re-sorted every few steps), so a wavefront's
// lanes come in runs of equal keys: the first lane of a run adds the run's
// length to the histogram and claims its slots in one atomic each.  Order
// inside a bucket follows the atomics (not stable).

// Runs of equal valid keys in the wavefront: bit l of *heads marks a lane
// that starts a run; returns the run length for such a lane.
__device__ __forceinline__ int wave_run(unsigned k, bool valid, unsigned long long *heads) {
  const int lane = threadIdx.x & 63;
  const unsigned prev = __shfl_up(k, 1, 64);
  const bool prev_valid = __shfl_up(valid ? 1 : 0, 1, 64) != 0;
  const bool head = valid && (lane == 0 || !prev_valid || prev != k);
  const unsigned long long hm = __ballot(head), invalid = __ballot(!valid);
  *heads = hm;
  // the run ends at the next head or invalid lane above this one
  const unsigned long long above = (hm | invalid) & (lane == 63 ? 0ULL : (~0ULL << (lane + 1)));
  return above ? (__ffsll((long long)above) - 1 - lane) : (64 - lane);
}

__global__ __launch_bounds__(256) void k_key_hist(const unsigned *keys, long long n, unsigned nkeys,
                                                  unsigned *count) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  const unsigned k = i < n ? keys[i] : 0xFFFFFFFFu;
  const bool valid = k < nkeys;
  unsigned long long heads;
  const int len = wave_run(k, valid, &heads);
  if (valid && ((heads >> (threadIdx.x & 63)) & 1ULL)) atomicAdd(count + k, (unsigned)len);
}

// Scan, phase 1: sums and occupied buckets of each 4096-bucket block.
constexpr int kScanPer = 16;                 // buckets per thread
constexpr int kScanBlock = 256 * kScanPer;   // buckets per workgroup

__global__ __launch_bounds__(256) void k_key_scan_blocks(const unsigned *count, unsigned nkeys,
                                                         unsigned long long *bsum, unsigned *bocc) {
  __shared__ unsigned long long ps[4];
  __shared__ unsigned po[4];
  const long long k0 = blockIdx.x * (long long)kScanBlock + threadIdx.x * (long long)kScanPer;
  unsigned long long sum = 0;
  unsigned occ = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const unsigned c = k0 + j < nkeys ? count[k0 + j] : 0u;
    sum += c;
    occ += c != 0u;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o, 64);
    occ += __shfl_xor(occ, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    ps[threadIdx.x >> 6] = sum;
    po[threadIdx.x >> 6] = occ;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bsum[blockIdx.x] = ps[0] + ps[1] + ps[2] + ps[3];
    bocc[blockIdx.x] = po[0] + po[1] + po[2] + po[3];
  }
}

// Scan, phase 2 (one workgroup of 1024 threads): exclusive prefix of the
// block sums in place; totals[0] = alive particles, totals[1] = occupied
// buckets.
__global__ __launch_bounds__(1024) void k_key_scan_top(unsigned long long *bsum, const unsigned *bocc,
                                                       long long nb, unsigned long long *totals) {
  __shared__ unsigned long long wsum[16];
  __shared__ unsigned long long wocc[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const long long per = (nb + 1023) / 1024;
  const long long b0 = t * per;
  unsigned long long s = 0, occ = 0;
  for (long long j = 0; j < per; ++j)
    if (b0 + j < nb) {
      s += bsum[b0 + j];
      occ += bocc[b0 + j];
    }
  // inclusive scan of s over the workgroup
  unsigned long long x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  unsigned long long oc = occ;
  for (int o = 32; o > 0; o >>= 1) oc += __shfl_xor(oc, o, 64);
  if (lane == 63) wsum[w] = x;
  if (lane == 0) wocc[w] = oc;
  __syncthreads();
  unsigned long long pre = 0, tot = 0, totocc = 0;
  for (int j = 0; j < 16; ++j) {
    if (j < w) pre += wsum[j];
    tot += wsum[j];
    totocc += wocc[j];
  }
  unsigned long long run = pre + x - s;  // exclusive prefix of this thread's first block
  for (long long j = 0; j < per; ++j)
    if (b0 + j < nb) {
      const unsigned long long v = bsum[b0 + j];
      bsum[b0 + j] = run;
      run += v;
    }
  if (t == 0) {
    totals[0] = tot;
    totals[1] = totocc;
  }
}

// Scan, phase 3: bucket starts (exclusive prefix) written over the counts.
__global__ __launch_bounds__(256) void k_key_scan_apply(unsigned *count, unsigned nkeys,
                                                        const unsigned long long *bsum) {
  __shared__ unsigned ws[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const long long k0 = blockIdx.x * (long long)kScanBlock + t * (long long)kScanPer;
  unsigned c[kScanPer], s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    c[j] = k0 + j < nkeys ? count[k0 + j] : 0u;
    s += c[j];
  }
  unsigned x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[w] = x;
  __syncthreads();
  unsigned pre = 0;
  for (int j = 0; j < w; ++j) pre += ws[j];
  unsigned run = (unsigned)bsum[blockIdx.x] + pre + x - s;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j)
    if (k0 + j < nkeys) {
      count[k0 + j] = run;
      run += c[j];
    }
}

// Scatter: particle i to the next free slot of its bucket; sorted keys and
// indices out.
__global__ __launch_bounds__(256) void k_key_scatter(const unsigned *keys, long long n, unsigned nkeys,
                                                     unsigned *cursor, unsigned *keys_out, unsigned *idx_out) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  const unsigned k = i < n ? keys[i] : 0xFFFFFFFFu;
  const bool valid = k < nkeys;
  unsigned long long heads;
  const int len = wave_run(k, valid, &heads);
  const int lane = threadIdx.x & 63;
  unsigned base = 0;
  if (valid && ((heads >> lane) & 1ULL)) base = atomicAdd(cursor + k, (unsigned)len);
  // the run's first lane: the highest head at or below this lane
  const unsigned long long below = heads & (lane == 63 ? ~0ULL : ((2ULL << lane) - 1));
  const int hl = below ? 63 - __clzll((long long)below) : lane;
  base = __shfl(base, hl, 64);
  if (valid) {
    const unsigned dst = base + (unsigned)(lane - hl);
    keys_out[dst] = k;
    idx_out[dst] = (unsigned)i;
  }
}

long long key_scan_blocks(unsigned nkeys) { return ((long long)nkeys + kScanBlock - 1) / kScanBlock; }

void launch_key_sort(const unsigned *keys, long long n, unsigned nkeys, unsigned *count, unsigned long long *bsum,
                     unsigned *bocc, unsigned long long *totals, unsigned *keys_out, unsigned *idx_out,
                     hipStream_t st) {
  const long long nb = key_scan_blocks(nkeys);
  const unsigned pgrid = (unsigned)((n + 255) / 256);
  if (n > 0) k_key_hist<<<pgrid, 256, 0, st>>>(keys, n, nkeys, count);
  k_key_scan_blocks<<<(unsigned)nb, 256, 0, st>>>(count, nkeys, bsum, bocc);
  k_key_scan_top<<<1, 1024, 0, st>>>(bsum, bocc, nb, totals);
  k_key_scan_apply<<<(unsigned)nb, 256, 0, st>>>(count, nkeys, bsum);
  if (n > 0) k_key_scatter<<<pgrid, 256, 0, st>>>(keys, n, nkeys, count, keys_out, idx_out);
}


// Sort key of a packed cell: with tiles = t > 0, cells are grouped in
// 2^t x 4 x 4 (2D: 2^t x 4) tiles, x1 fastest inside a tile, so that a chunk
// of consecutive particles covers a compact 3D region (its LDS box stays
// small when the particles fill the grid, as a plasma does).  Tiles count x1
// from the moving window's first cell, not from the ring buffer's first
// storage column: a tile then never holds both ends of the window (whose
// box would span it), and after later shifts its cells stay contiguous.
// tiles = 0: the packed index itself.  Both are one-to-one on cells.
template <typename Real>
__global__ void k_sort_keys(Geo g, Particles<Real> p, int tiles, unsigned *keys, unsigned *idx) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const int c = p.cell[i];
  unsigned k = 0xFFFFFFFFu;
  if (c >= 0) {
    k = (unsigned)c;
    if (tiles > 0) {
      int s1, c2, c3;
      unpack_cell(g, c, s1, c2, c3);
      s1 -= g.ws_mod;  // window x1
      if (s1 < 0) s1 += g.n1;
      const unsigned w1 = 1u << tiles;
      const unsigned nt1 = ((unsigned)g.n1 + w1 - 1) >> tiles, nt2 = (unsigned)(g.n2 + 3) >> 2;
      const unsigned tile = ((unsigned)(c3 >> 2) * nt2 + (unsigned)(c2 >> 2)) * nt1 + ((unsigned)s1 >> tiles);
      const unsigned local = (((unsigned)(c3 & 3) * 4 + (unsigned)(c2 & 3)) << tiles) + ((unsigned)s1 & (w1 - 1));
      k = tile * ((g.n3 > 1 ? 16u : 4u) << tiles) + local;
    }
  }
  keys[i] = k;
  idx[i] = (unsigned)i;
}

template <typename Real>
__global__ void k_permute(Particles<Real> src, Particles<Real> dst, const int *id_src, int *id_dst,
                          const unsigned *perm, int ndim, const unsigned long long *count) {
  const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (j >= src.n || (count && (unsigned long long)j >= *count)) return;
  const long long i = perm[j];
  const int c = src.cell[i];
  dst.cell[j] = c;
  dst.o1[j] = src.o1[i];
  dst.o2[j] = src.o2[i];
  if (ndim == 3) dst.o3[j] = src.o3[i];
  dst.u1[j] = src.u1[i];
  dst.u2[j] = src.u2[i];
  dst.u3[j] = src.u3[i];
  id_dst[j] = id_src[i];
}

// In a sorted key array: the number of distinct alive cells (density
// estimate) and the number of alive particles, written by the last alive
// slot (dropped particles sort last; both counters zero beforehand).  A
// counter that every wavefront hits serializes in L2 (65536 atomics on one
// address took ~0.8 ms), so the runs are summed per workgroup over a bounded
// grid and the alive count is not accumulated at all.  4096 workgroups (16
// per CU) keep enough loads in flight (512 read 2.7e8 keys at 0.5 TB/s).
constexpr int kRunsBlocks = 4096;

__global__ __launch_bounds__(256) void k_count_runs(const unsigned *keys, long long n, unsigned long long *runs,
                                                    unsigned long long *alive) {
  __shared__ unsigned long long part[4];
  unsigned long long cnt = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const unsigned k = keys[i];
    if (k == 0xFFFFFFFFu) continue;
    if (i == 0 || keys[i - 1] != k) ++cnt;
    if (i + 1 == n || keys[i + 1] == 0xFFFFFFFFu) *alive = (unsigned long long)(i + 1);
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long tot = part[0] + part[1] + part[2] + part[3];
    if (tot) atomicAdd(runs, tot);
  }
}

void launch_count_runs(const unsigned *keys, long long n, unsigned long long *runs, unsigned long long *alive,
                       hipStream_t st) {
  if (n <= 0) return;
  const long long need = (n + 255) / 256;
  k_count_runs<<<(unsigned)(need < kRunsBlocks ? need : kRunsBlocks), 256, 0, st>>>(keys, n, runs, alive);
}

template <typename Real>
void launch_sort_keys(const Geo &g, const Particles<Real> &p, int tiles, unsigned *keys, unsigned *idx,
                      hipStream_t st) {
  if (p.n <= 0) return;
  k_sort_keys<Real><<<(unsigned)((p.n + 255) / 256), 256, 0, st>>>(g, p, tiles, keys, idx);
}

template <typename Real>
void launch_permute(const Particles<Real> &src, const Particles<Real> &dst, const int *id_src, int *id_dst,
                    const unsigned *perm, int ndim, hipStream_t st, const unsigned long long *count) {
  if (src.n <= 0) return;
  k_permute<Real><<<(unsigned)((src.n + 255) / 256), 256, 0, st>>>(src, dst, id_src, id_dst, perm, ndim, count);
}

#define RELPIC_INST_PART(Real)                                                                                   \
  template void launch_push_deposit<Real>(int, const Geo &, const Fields<Real> &, const HalfB<Real> &,          \
                                          const Particles<Real> &, const PushParams<Real> &, const PushChunks &, \
                                          bool, bool, JBox *, int *, hipStream_t);                               \
  template void launch_sort_keys<Real>(const Geo &, const Particles<Real> &, int, unsigned *, unsigned *,        \
                                       hipStream_t);                                                             \
  template void launch_permute<Real>(const Particles<Real> &, const Particles<Real> &, const int *, int *,      \
                                     const unsigned *, int, hipStream_t, const unsigned long long *);

RELPIC_INST_PART(float)
RELPIC_INST_PART(double)

}  // namespace relpic
