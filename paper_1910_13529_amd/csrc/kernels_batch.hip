// Batched many-run kernels.  Each launch covers every run of the batch: the
// field kernels walk a table of (run, x1 segment, row range) tiles, the
// particle kernel a table of (run species, chunk) entries, and the small
// per-box kernels take a fixed number of workgroups per run.  The per-tile
// and per-chunk work is the device code of the single-run kernels, so a run
// in a batch computes what it computes alone.
#include "batch_kernels.h"
#include "field_tiles.h"
#include "particle_chunk.h"

namespace relpic {

constexpr int kStage = stage_pitch<kBatchSeg>();
constexpr int kBoxWorkgroups = 4;  // workgroups per run of the deposit-box kernels

// The tiles [band * per, (band + 1) * per) of the table go to the workgroups
// on XCD `band` (workgroup b runs on XCD b mod 8), which sweep them with a
// stride equal to their number, so neighbouring rows of one run share an L2.
// A grid of 8 * per workgroups takes one tile each; a smaller grid loops.
__device__ __forceinline__ void band_range(int ntiles, int &first, int &end, int &step) {
  const int band = (int)(blockIdx.x % kNumXcd);
  const int per = (ntiles + kNumXcd - 1) / kNumXcd;
  first = band * per + (int)(blockIdx.x / kNumXcd);
  end = min((band + 1) * per, ntiles);
  step = (int)(gridDim.x / kNumXcd);
}

template <typename Real>
__global__ __launch_bounds__(kBatchSeg) void k_batch_curl_e(const BatchRun<Real> *__restrict__ runs,
                                                            const BatchTile *__restrict__ tiles, int ntiles, int bin,
                                                            int which) {
  __shared__ Real s2[kStage], s3[kStage];
  int t, end, step;
  band_range(ntiles, t, end, step);
  for (; t < end; t += step) {
    const BatchTile tl = tiles[t];
    const BatchRun<Real> &r = runs[tl.run];
    Real *const *Bi = r.B[bin];
    Real *const *Bo = r.B[bin ^ 1];
    const Axial<Real> &ax = r.ax[which];
    // the branch is uniform over the workgroup; each call ends with a barrier
    if (r.M == 1)
      curl_e_rows<Real, 1, kBatchSeg>(r.g, r.E1, r.E2, r.E3, Bi[0], Bi[1], Bi[2], Bo[0], Bo[1], Bo[2], ax,
                                      r.h2[which], tl.l0, tl.r0, tl.r1, s2, s3);
    else if (r.M == 16)
      curl_e_rows<Real, 16, kBatchSeg>(r.g, r.E1, r.E2, r.E3, Bi[0], Bi[1], Bi[2], Bo[0], Bo[1], Bo[2], ax,
                                       r.h2[which], tl.l0, tl.r0, tl.r1, s2, s3);
    else
      curl_e_rows<Real, 0, kBatchSeg>(r.g, r.E1, r.E2, r.E3, Bi[0], Bi[1], Bi[2], Bo[0], Bo[1], Bo[2], ax,
                                      r.h2[which], tl.l0, tl.r0, tl.r1, s2, s3);
  }
}

template <typename Real>
__global__ __launch_bounds__(kBatchSeg) void k_batch_curl_b(const BatchRun<Real> *__restrict__ runs,
                                                            const BatchTile *__restrict__ tiles, int ntiles,
                                                            int bsel) {
  __shared__ Real s2[kStage], s3[kStage];
  int t, end, step;
  band_range(ntiles, t, end, step);
  for (; t < end; t += step) {
    const BatchTile tl = tiles[t];
    const BatchRun<Real> &r = runs[tl.run];
    Real *const *B = r.B[bsel];
    if (r.M == 1)
      curl_b_rows<Real, 1, kBatchSeg>(r.g, r.E1, r.E2, r.E3, B[0], B[1], B[2], r.ax[0], r.h2[0], tl.l0, tl.r0, tl.r1,
                                      s2, s3);
    else if (r.M == 16)
      curl_b_rows<Real, 16, kBatchSeg>(r.g, r.E1, r.E2, r.E3, B[0], B[1], B[2], r.ax[0], r.h2[0], tl.l0, tl.r0,
                                       tl.r1, s2, s3);
    else
      curl_b_rows<Real, 0, kBatchSeg>(r.g, r.E1, r.E2, r.E3, B[0], B[1], B[2], r.ax[0], r.h2[0], tl.l0, tl.r0, tl.r1,
                                      s2, s3);
  }
}

template <typename Real>
__global__ __launch_bounds__(kPushBlock) void k_batch_push(const BatchRun<Real> *__restrict__ runs,
                                                           const BatchPart<Real> *__restrict__ parts,
                                                           const BatchChunk *__restrict__ chunks, int bnew,
                                                           JBox *chunkbox, int *err) {
  __shared__ __align__(16) unsigned char tile_raw[kTileBytes];
  __shared__ int box[kChunkBoxInts];
  const BatchChunk c = chunks[blockIdx.x];
  const BatchPart<Real> &pd = parts[c.part];
  const BatchRun<Real> &r = runs[pd.run];
  Fields<Real> f;
  f.E1 = r.E1;
  f.E2 = r.E2;
  f.E3 = r.E3;
  f.B1 = r.B[bnew][0];
  f.B2 = r.B[bnew][1];
  f.B3 = r.B[bnew][2];
  f.J1 = r.J1;
  f.J2 = r.J2;
  f.J3 = r.J3;
  f.J1c = r.J1c;
  const HalfB<Real> Bh{r.B[bnew ^ 1][0], r.B[bnew ^ 1][1], r.B[bnew ^ 1][2]};
  const long long c0 = c.chunk * (long long)kPushBlock * pd.K;
  push_chunk<Real, 2>(r.g, f, Bh, pd.p, pd.q, c0, c0 + (long long)kPushBlock * pd.K, chunkbox + blockIdx.x, err,
                      tile_raw, box);
}

// box[run] = union of the run's chunk boxes (one wavefront per run)
template <typename Real>
__global__ __launch_bounds__(64) void k_batch_merge(const BatchRun<Real> *__restrict__ runs,
                                                    const JBox *__restrict__ chunkbox, JBox *box) {
  const BatchRun<Real> &r = runs[blockIdx.x];
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {-INT_MAX, -INT_MAX, -INT_MAX};
  for (int k = threadIdx.x; k < r.nchunk; k += 64) {
    const JBox &b = chunkbox[r.chunk0 + k];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], b.lo[d]);
      hi[d] = max(hi[d], b.hi[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
      hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
    }
  if (threadIdx.x == 0)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      box[blockIdx.x].lo[d] = lo[d];
      box[blockIdx.x].hi[d] = hi[d];
    }
}

template <typename Real>
__global__ __launch_bounds__(256) void k_batch_jcorr(const BatchRun<Real> *__restrict__ runs,
                                                     const JBox *__restrict__ box) {
  const int run = (int)(blockIdx.x / kBoxWorkgroups);
  const BatchRun<Real> &r = runs[run];
  if (r.M == 1) return;
  jcorr_box(r.g, r.J1, r.J1c, r.taps, r.ng, box[run], (long long)(blockIdx.x % kBoxWorkgroups) * 256 + threadIdx.x,
            (long long)kBoxWorkgroups * 256);
}

template <typename Real>
__global__ __launch_bounds__(256) void k_batch_add_j(const BatchRun<Real> *__restrict__ runs,
                                                     const JBox *__restrict__ box) {
  const int run = (int)(blockIdx.x / kBoxWorkgroups);
  const BatchRun<Real> &r = runs[run];
  const bool corr = r.M > 1;
  add_j_box(r.g, r.E1, r.E2, r.E3, r.J1, r.J2, r.J3, corr ? r.J1c : r.J1, r.dt, box[run], corr ? r.ng : 0,
            (long long)(blockIdx.x % kBoxWorkgroups) * 256 + threadIdx.x, (long long)kBoxWorkgroups * 256);
}

// ---- batch-wide sort ------------------------------------------------------------

// index d of the particle set holding batch slot i: base[d] <= i < base[d + 1]
__device__ __forceinline__ int part_of(const long long *base, int nparts, long long i) {
  int lo = 0, hi = nparts;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename Real>
__global__ void k_batch_sort_keys(const BatchPart<Real> *__restrict__ parts, int nparts,
                                  const long long *__restrict__ base, long long ntot, int cbits, unsigned *keys,
                                  unsigned *idx) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  const int d = part_of(base, nparts, i);
  const int c = parts[d].p.cell[i - base[d]];
  const unsigned dead = (1u << cbits) - 1u;
  keys[i] = ((unsigned)d << cbits) | (c < 0 ? dead : (unsigned)c);
  idx[i] = (unsigned)i;
}

template <typename Real>
__global__ void k_batch_permute(const BatchPart<Real> *__restrict__ parts, long long ntot, int cbits,
                                const unsigned *__restrict__ keys, const unsigned *__restrict__ idx,
                                unsigned long long *runs_out) {
  const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (j >= ntot) return;
  const unsigned key = keys[j];
  const int d = (int)(key >> cbits);
  const BatchPart<Real> &pd = parts[d];
  const long long src = (long long)idx[j] - pd.base, dst = j - pd.base;
  pd.p2.cell[dst] = pd.p.cell[src];
  pd.p2.o1[dst] = pd.p.o1[src];
  pd.p2.o2[dst] = pd.p.o2[src];
  pd.p2.u1[dst] = pd.p.u1[src];
  pd.p2.u2[dst] = pd.p.u2[src];
  pd.p2.u3[dst] = pd.p.u3[src];
  pd.id2[dst] = pd.id[src];
  const unsigned dead = (1u << cbits) - 1u;
  if (runs_out && (key & dead) != dead && (dst == 0 || keys[j - 1] != key)) atomicAdd(runs_out + d, 1ULL);
}

template <typename Real>
__global__ void k_batch_copy_back(const BatchPart<Real> *__restrict__ parts, int nparts,
                                  const long long *__restrict__ base, long long ntot) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  const int d = part_of(base, nparts, i);
  const BatchPart<Real> &pd = parts[d];
  const long long k = i - base[d];
  pd.p.cell[k] = pd.p2.cell[k];
  pd.p.o1[k] = pd.p2.o1[k];
  pd.p.o2[k] = pd.p2.o2[k];
  pd.p.u1[k] = pd.p2.u1[k];
  pd.p.u2[k] = pd.p2.u2[k];
  pd.p.u3[k] = pd.p2.u3[k];
  pd.id[k] = pd.id2[k];
}

// ---- launchers ---------------------------------------------------------------

template <typename Real>
void launch_batch_curl_e(const BatchRun<Real> *runs, const BatchTile *tiles, int ntiles, int grid, int bin, int which,
                         hipStream_t st) {
  k_batch_curl_e<Real><<<grid, kBatchSeg, 0, st>>>(runs, tiles, ntiles, bin, which);
}

template <typename Real>
void launch_batch_curl_b(const BatchRun<Real> *runs, const BatchTile *tiles, int ntiles, int grid, int bsel,
                         hipStream_t st) {
  k_batch_curl_b<Real><<<grid, kBatchSeg, 0, st>>>(runs, tiles, ntiles, bsel);
}

template <typename Real>
void launch_batch_push(const BatchRun<Real> *runs, int nruns, const BatchPart<Real> *parts, const BatchChunk *chunks,
                       int nchunks, int bnew, JBox *chunkbox, JBox *box, int *err, hipStream_t st) {
  if (nchunks > 0) k_batch_push<Real><<<nchunks, kPushBlock, 0, st>>>(runs, parts, chunks, bnew, chunkbox, err);
  k_batch_merge<Real><<<nruns, 64, 0, st>>>(runs, chunkbox, box);
}

template <typename Real>
void launch_batch_jcorr(const BatchRun<Real> *runs, int nruns, const JBox *box, hipStream_t st) {
  k_batch_jcorr<Real><<<nruns * kBoxWorkgroups, 256, 0, st>>>(runs, box);
}

template <typename Real>
void launch_batch_add_j(const BatchRun<Real> *runs, int nruns, const JBox *box, hipStream_t st) {
  k_batch_add_j<Real><<<nruns * kBoxWorkgroups, 256, 0, st>>>(runs, box);
}

template <typename Real>
void launch_batch_sort_keys(const BatchPart<Real> *parts, int nparts, const long long *base, long long ntot, int cbits,
                            unsigned *keys, unsigned *idx, hipStream_t st) {
  if (ntot <= 0) return;
  k_batch_sort_keys<Real><<<(unsigned)((ntot + 255) / 256), 256, 0, st>>>(parts, nparts, base, ntot, cbits, keys, idx);
}

template <typename Real>
void launch_batch_permute(const BatchPart<Real> *parts, long long ntot, int cbits, const unsigned *keys,
                          const unsigned *idx, unsigned long long *runs_out, hipStream_t st) {
  if (ntot <= 0) return;
  k_batch_permute<Real><<<(unsigned)((ntot + 255) / 256), 256, 0, st>>>(parts, ntot, cbits, keys, idx, runs_out);
}

template <typename Real>
void launch_batch_copy_back(const BatchPart<Real> *parts, int nparts, const long long *base, long long ntot,
                            hipStream_t st) {
  if (ntot <= 0) return;
  k_batch_copy_back<Real><<<(unsigned)((ntot + 255) / 256), 256, 0, st>>>(parts, nparts, base, ntot);
}

#define RELPIC_INST_BATCH(Real)                                                                                   \
  template void launch_batch_curl_e<Real>(const BatchRun<Real> *, const BatchTile *, int, int, int, int,          \
                                          hipStream_t);                                                          \
  template void launch_batch_curl_b<Real>(const BatchRun<Real> *, const BatchTile *, int, int, int, hipStream_t); \
  template void launch_batch_push<Real>(const BatchRun<Real> *, int, const BatchPart<Real> *, const BatchChunk *, \
                                        int, int, JBox *, JBox *, int *, hipStream_t);                           \
  template void launch_batch_jcorr<Real>(const BatchRun<Real> *, int, const JBox *, hipStream_t);                 \
  template void launch_batch_add_j<Real>(const BatchRun<Real> *, int, const JBox *, hipStream_t);                 \
  template void launch_batch_sort_keys<Real>(const BatchPart<Real> *, int, const long long *, long long, int,     \
                                             unsigned *, unsigned *, hipStream_t);                               \
  template void launch_batch_permute<Real>(const BatchPart<Real> *, long long, int, const unsigned *,             \
                                           const unsigned *, unsigned long long *, hipStream_t);                 \
  template void launch_batch_copy_back<Real>(const BatchPart<Real> *, int, const long long *, long long, hipStream_t);

RELPIC_INST_BATCH(float)
RELPIC_INST_BATCH(double)

}  // namespace relpic
