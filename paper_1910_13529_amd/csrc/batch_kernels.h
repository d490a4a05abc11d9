// Batched many-run path: device tables and launch entry points (internal to
// relpic).  Many independent 2D periodic runs, each with its own grid, time
// step, operator and particles, advance together: every phase of the step is
// one launch over all runs, driven by host-built tables.
#pragma once

#include "kernels.h"

namespace relpic {

// Field tiles: a kBatchSeg-cell x1 segment (one thread per cell) marching
// through kShapeRows[shape] consecutive x2 rows.
constexpr int kBatchSeg = 128;
constexpr int kNumShapes = 3;
constexpr int kShapeRows[kNumShapes] = {4, 8, 16};

// Per-run constants and device pointers (one entry per run).
template <typename Real>
struct BatchRun {
  Geo g;
  Real *E1, *E2, *E3, *J1, *J2, *J3, *J1c;
  Real *B[2][3];      // the two B buffers (slots); the host tracks which holds what
  const Real *taps;   // J1 correction FIR g_0..g_ng (M > 1)
  int ng;
  int M;
  int shape;          // field tile shape
  int chunk0, nchunk; // the run's entries in the push chunk table
  Axial<Real> ax[3];  // C_l f dt / dx1 for f = 1, -1/2, +1/2
  Real h2[3];         // f dt / dx2, same factors
  Real dt;
};

// Per (run, species) particle arrays and push constants.
template <typename Real>
struct BatchPart {
  Particles<Real> p;   // primary arrays (what the push reads and writes)
  Particles<Real> p2;  // secondary arrays (sort target)
  int *id, *id2;
  PushParams<Real> q;
  int run, K;
  long long base;      // first slot of these particles in the batch-wide sort arrays
};

struct BatchTile {
  int run, l0, r0, r1;  // x1 segment start, rows r0 .. r1 - 1
};

struct BatchChunk {
  int part, chunk;
};

// Field tables selected per launch: which = 0 full step, 1 the -dt/2
// half step, 2 the +dt/2 half step; workgroups of kBatchSeg threads.
// Bout = Bin - curl+ E with Bin = slot `bin` and Bout = slot 1 - bin.
template <typename Real>
void launch_batch_curl_e(const BatchRun<Real> *runs, const BatchTile *tiles, int ntiles, int grid, int bin, int which,
                         hipStream_t st);
// E += dt curl- B with B = slot `bsel`
template <typename Real>
void launch_batch_curl_b(const BatchRun<Real> *runs, const BatchTile *tiles, int ntiles, int grid, int bsel,
                         hipStream_t st);
// gather (E, B^n = average of the slots) + push + deposit; slot `bnew` holds
// B^{n+1/2}.  Followed by the per-run merge of the chunk boxes into box[run].
template <typename Real>
void launch_batch_push(const BatchRun<Real> *runs, int nruns, const BatchPart<Real> *parts, const BatchChunk *chunks,
                       int nchunks, int bnew, JBox *chunkbox, JBox *box, int *err, hipStream_t st);
// J1 correction inside each customized run's deposit box
template <typename Real>
void launch_batch_jcorr(const BatchRun<Real> *runs, int nruns, const JBox *box, hipStream_t st);
// E -= dt J (J1 corrected for M > 1) inside each run's box, J cleared there
template <typename Real>
void launch_batch_add_j(const BatchRun<Real> *runs, int nruns, const JBox *box, hipStream_t st);

// Batch-wide cell sort: keys (part << cbits | cell) over all particles, then
// a gather into the secondary arrays and a copy back, so the primary arrays
// keep their addresses.  runs_out[part] += number of occupied cells (if set).
template <typename Real>
void launch_batch_sort_keys(const BatchPart<Real> *parts, int nparts, const long long *base, long long ntot, int cbits,
                            unsigned *keys, unsigned *idx, hipStream_t st);
template <typename Real>
void launch_batch_permute(const BatchPart<Real> *parts, long long ntot, int cbits, const unsigned *keys,
                          const unsigned *idx, unsigned long long *runs_out, hipStream_t st);
template <typename Real>
void launch_batch_copy_back(const BatchPart<Real> *parts, int nparts, const long long *base, long long ntot,
                            hipStream_t st);

hipError_t sort_pairs_bits(void *temp, size_t &temp_bytes, const unsigned *keys_in, unsigned *keys_out,
                           const unsigned *idx_in, unsigned *idx_out, long long n, int end_bit, hipStream_t st);

}  // namespace relpic
