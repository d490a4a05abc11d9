// Batched many-run engine and its C ABI.  A batch owns one relpic_sim per run
// (so particles, fields, diagnostics and reads go through the single-run
// calls) and advances all of them together: each phase of a step is one
// launch over every run, driven by device tables of per-run constants, field
// tiles and push chunks.  Steps between particle sorts are recorded once into
// a HIP graph and replayed.
//
// B is kept in two slots per run.  Between calls slot `canon` holds B^n; a
// call opens with the -dt/2 half step into the other slot, alternates the
// slots every step and closes with the +dt/2 half step, as the single-run
// engine does with its two buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "batch_kernels.h"
#include "engine.h"

using namespace relpic;
using namespace relpic_host;

struct relpic_batch {
  relpic_precision prec = RELPIC_FP32;
  size_t esz = 4;
  relpic_device dev{};
  hipStream_t st = nullptr;
  std::vector<relpic_sim *> runs;
  std::vector<std::pair<void *, size_t>> owned;  // device allocations of the batch itself
  // device tables
  void *d_runs = nullptr;
  void *d_parts = nullptr;
  size_t parts_cap = 0;
  long long *d_base = nullptr;
  size_t base_cap = 0;
  BatchTile *d_tiles = nullptr;
  size_t tiles_cap = 0;
  BatchChunk *d_chunks = nullptr;
  size_t chunks_cap = 0;
  JBox *d_chunkbox = nullptr;
  size_t chunkbox_cap = 0;
  JBox *d_box = nullptr;
  int *err = nullptr;
  unsigned long long *d_count = nullptr;  // occupied cells per particle set (sort)
  size_t count_cap = 0;
  unsigned *keys = nullptr, *keys2 = nullptr, *idx = nullptr, *idx2 = nullptr;
  long long sort_cap = 0;
  void *sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  int ntiles = 0, nchunks = 0, nparts = 0;
  long long ntot = 0;
  int cbits = 1, kbits = 1;
  bool any_custom = false;
  // tiling
  std::vector<int> shape;  // per run
  int grid_wg = 0;         // field-kernel workgroups (0: one per tile)
  // stepping state
  int canon = 0;
  long long bstep = 0;
  long long sorted_at = -1;  // bstep of the last sort
  int graph_steps = 20;
  hipStream_t cap_st = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  bool prepared = false;
  std::vector<const void *> sig;  // sub-simulation state at the last table build
  std::vector<void *> slot[2];    // per run x 3: the two B slots
};

namespace {

constexpr int kSortEvery = 20;  // particle sort interval when graphs are off

void *balloc(relpic_batch *b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void *p = nullptr;
  if (b->dev.alloc)
    p = b->dev.alloc(bytes, b->dev.user);
  else if (hipMalloc(&p, bytes) != hipSuccess)
    p = nullptr;
  if (p) b->owned.emplace_back(p, bytes);
  return p;
}

void bfree(relpic_batch *b, void *p) {
  if (!p) return;
  for (size_t i = 0; i < b->owned.size(); ++i)
    if (b->owned[i].first == p) {
      if (b->dev.free)
        b->dev.free(p, b->dev.user);
      else if (!b->dev.alloc)
        (void)hipFree(p);
      b->owned.erase(b->owned.begin() + (long)i);
      return;
    }
}

// grow a device buffer to at least `need` elements of `elem` bytes
template <typename T>
bool ensure(relpic_batch *b, T *&p, size_t &cap, size_t need, size_t elem = sizeof(T)) {
  if (need <= cap && p) return true;
  bfree(b, (void *)p);
  const size_t n = std::max<size_t>(need, 1);
  p = (T *)balloc(b, n * elem);
  cap = p ? n : 0;
  return p != nullptr;
}

void drop_graphs(relpic_batch *b) {
  for (int k = 0; k < 2; ++k) {
    if (b->gexec[k]) (void)hipGraphExecDestroy(b->gexec[k]);
    if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
    b->gexec[k] = nullptr;
    b->graph[k] = nullptr;
  }
}

int bits_for(long long v) {  // smallest k with 2^k > v
  int k = 0;
  while (k < 62 && (1LL << k) <= v) ++k;
  return k;
}

long long shape_tiles(const relpic_sim *s, int shape) {
  const long long nseg = (s->n[0] + kBatchSeg - 1) / kBatchSeg;
  const long long nrow = (s->n[1] + kShapeRows[shape] - 1) / kShapeRows[shape];
  return nseg * nrow;
}

// default tile shape before any autotuning: the middle row count
constexpr int kDefaultShape = 1;

// state of the sub-simulations that the device tables depend on
std::vector<const void *> signature(const relpic_batch *b) {
  std::vector<const void *> v;
  for (const relpic_sim *s : b->runs) {
    for (int k = 0; k < 10; ++k)
      if (k < 3 || k > 5) v.push_back(s->F[k]);
    v.push_back((const void *)(intptr_t)s->sp.size());
    for (const Species &sp : s->sp) {
      v.push_back((const void *)(intptr_t)sp.n);
      v.push_back((const void *)(intptr_t)(sp.dirty ? 1 : 0));
      v.push_back(sp.cell);
      v.push_back(sp.cell2);
      v.push_back(sp.id);
      for (int d = 0; d < 3; ++d) {
        v.push_back(sp.o[d]);
        v.push_back(sp.u[d]);
      }
    }
  }
  return v;
}

bool slots_match(const relpic_batch *b) {
  for (size_t r = 0; r < b->runs.size(); ++r)
    for (int d = 0; d < 3; ++d)
      if (b->runs[r]->F[3 + d] != b->slot[b->canon][3 * r + d] || b->runs[r]->Bx[d] != b->slot[1 - b->canon][3 * r + d])
        return false;
  return true;
}

template <typename Real>
relpic_status build_tiles(relpic_batch *b) {
  // tiles in run order: the XCD bands then cut the table into contiguous
  // ranges with a balanced mix of cheap (Yee) and costly (customized) runs
  std::vector<BatchTile> t;
  for (int r = 0; r < (int)b->runs.size(); ++r) {
    const relpic_sim *s = b->runs[r];
    const int rows = kShapeRows[b->shape[r]];
    for (int r0 = 0; r0 < s->n[1]; r0 += rows) {
      const int r1 = std::min(r0 + rows, (int)s->n[1]);
      for (int l0 = 0; l0 < s->n[0]; l0 += kBatchSeg) t.push_back(BatchTile{r, l0, r0, r1});
    }
  }
  if (t.size() >= (size_t)INT32_MAX / 2) return fail(RELPIC_EINVAL, "batch: too many field tiles");
  if (!ensure(b, b->d_tiles, b->tiles_cap, t.size())) return fail(RELPIC_ENOMEM, "batch: tile table allocation failed");
  HIP_OK(hipMemcpyAsync(b->d_tiles, t.data(), sizeof(BatchTile) * t.size(), hipMemcpyHostToDevice, b->st));
  b->ntiles = (int)t.size();
  // per-run shape lives in the run table
  for (size_t r = 0; r < b->runs.size(); ++r) {
    const size_t off = sizeof(BatchRun<Real>) * r + offsetof(BatchRun<Real>, shape);
    HIP_OK(hipMemcpyAsync((char *)b->d_runs + off, &b->shape[r], sizeof(int), hipMemcpyHostToDevice, b->st));
  }
  HIP_OK(hipStreamSynchronize(b->st));
  drop_graphs(b);
  return RELPIC_OK;
}

int field_grid(const relpic_batch *b) {
  if (b->grid_wg > 0) return b->grid_wg;
  return (b->ntiles + 7) / 8 * 8;
}

// Sort every particle set by cell (batch-wide radix sort on part << cbits |
// cell).  With `count`, also pick each set's push chunk size from its
// particles per occupied cell (synchronizes).
template <typename Real>
relpic_status sort_all(relpic_batch *b, std::vector<BatchPart<Real>> *hparts) {
  if (b->ntot <= 1) return RELPIC_OK;
  launch_batch_sort_keys<Real>((const BatchPart<Real> *)b->d_parts, b->nparts, b->d_base, b->ntot, b->cbits, b->keys,
                               b->idx, b->st);
  size_t need = 0;
  HIP_OK(sort_pairs_bits(nullptr, need, b->keys, b->keys2, b->idx, b->idx2, b->ntot, b->cbits + b->kbits, b->st));
  if (need > b->sort_tmp_bytes || !b->sort_tmp) {
    bfree(b, b->sort_tmp);
    b->sort_tmp = balloc(b, need);
    if (!b->sort_tmp) return fail(RELPIC_ENOMEM, "batch sort: temporary storage allocation failed");
    b->sort_tmp_bytes = need;
  }
  HIP_OK(sort_pairs_bits(b->sort_tmp, need, b->keys, b->keys2, b->idx, b->idx2, b->ntot, b->cbits + b->kbits, b->st));
  if (hparts) HIP_OK(hipMemsetAsync(b->d_count, 0, sizeof(unsigned long long) * b->nparts, b->st));
  launch_batch_permute<Real>((const BatchPart<Real> *)b->d_parts, b->ntot, b->cbits, b->keys2, b->idx2,
                             hparts ? b->d_count : nullptr, b->st);
  launch_batch_copy_back<Real>((const BatchPart<Real> *)b->d_parts, b->nparts, b->d_base, b->ntot, b->st);
  HIP_OK(hipGetLastError());
  if (hparts) {
    std::vector<unsigned long long> cnt(b->nparts);
    HIP_OK(hipMemcpyAsync(cnt.data(), b->d_count, sizeof(unsigned long long) * b->nparts, hipMemcpyDeviceToHost,
                          b->st));
    HIP_OK(hipStreamSynchronize(b->st));
    for (int d = 0; d < b->nparts; ++d) {
      BatchPart<Real> &pd = (*hparts)[d];
      const double ppc = cnt[d] ? (double)pd.p.n / (double)cnt[d] : 0.0;
      pd.K = ppc >= 512.0 ? 8 : (ppc >= 64.0 ? 4 : (ppc >= 16.0 ? 2 : 1));
    }
  }
  return RELPIC_OK;
}

// Build every device table from the sub-simulations, sort the particles.
template <typename Real>
relpic_status prepare(relpic_batch *b) {
  const int nr = (int)b->runs.size();
  for (relpic_sim *s : b->runs) {
    if (s->ndim != 2 || s->grid.bc1 != RELPIC_BC_PERIODIC)
      return fail(RELPIC_ESTATE, "batch: runs must stay 2D and periodic");
    for (const Species &sp : s->sp)
      if (sp.inject) return fail(RELPIC_ESTATE, "batch: injection is not supported in a batch");
  }
  drop_graphs(b);
  // run table; slot 0 = the current B^n buffers
  b->canon = 0;
  for (int k = 0; k < 2; ++k) b->slot[k].assign(3 * nr, nullptr);
  std::vector<BatchRun<Real>> hr(nr);
  b->any_custom = false;
  long long maxN = 0;
  for (int r = 0; r < nr; ++r) {
    relpic_sim *s = b->runs[r];
    BatchRun<Real> &R = hr[r];
    std::memset((void *)&R, 0, sizeof(R));
    R.g = make_geo(s);
    const Fields<Real> f = fields<Real>(s);
    R.E1 = f.E1;
    R.E2 = f.E2;
    R.E3 = f.E3;
    R.J1 = f.J1;
    R.J2 = f.J2;
    R.J3 = f.J3;
    R.J1c = f.J1c;
    for (int d = 0; d < 3; ++d) {
      R.B[0][d] = (Real *)s->F[3 + d];
      R.B[1][d] = (Real *)s->Bx[d];
      b->slot[0][3 * r + d] = s->F[3 + d];
      b->slot[1][3 * r + d] = s->Bx[d];
    }
    R.taps = (const Real *)s->taps;
    R.ng = s->ng;
    R.M = s->M;
    R.shape = b->shape[r];
    const double dt = s->grid.dt;
    const double fac[3] = {1.0, -0.5, 0.5};
    for (int k = 0; k < 3; ++k) {
      R.ax[k] = axial_scaled<Real>(s, fac[k] * dt);
      R.h2[k] = (Real)(fac[k] * dt / s->dx[1]);
    }
    R.dt = (Real)dt;
    b->any_custom = b->any_custom || s->M > 1;
    maxN = std::max(maxN, s->N);
  }
  // particle sets
  std::vector<BatchPart<Real>> hp;
  std::vector<long long> base(1, 0);
  for (int r = 0; r < nr; ++r) {
    relpic_sim *s = b->runs[r];
    for (Species &sp : s->sp) {
      if (sp.n <= 0) continue;
      BatchPart<Real> P;
      std::memset((void *)&P, 0, sizeof(P));
      P.p = parts<Real>(sp);
      P.p2 = P.p;
      P.p2.cell = sp.cell2;
      P.p2.o1 = (Real *)sp.o2[0];
      P.p2.o2 = (Real *)sp.o2[1];
      P.p2.o3 = (Real *)sp.o2[2];
      P.p2.u1 = (Real *)sp.u2[0];
      P.p2.u2 = (Real *)sp.u2[1];
      P.p2.u3 = (Real *)sp.u2[2];
      P.id = sp.id;
      P.id2 = sp.id2;
      P.q = push_params<Real>(s, sp, 0);
      P.run = r;
      P.K = sp.K;
      P.base = base.back();
      hp.push_back(P);
      base.push_back(base.back() + sp.n);
    }
  }
  b->nparts = (int)hp.size();
  b->ntot = base.back();
  if (b->ntot >= (1LL << 32)) return fail(RELPIC_EINVAL, "batch: more than 2^32 particles");
  b->cbits = std::max(1, bits_for(maxN));
  b->kbits = bits_for(std::max(0, b->nparts - 1));
  if (b->cbits + b->kbits > 32) return fail(RELPIC_EINVAL, "batch: sort key exceeds 32 bits (runs x cells too large)");
  if (!b->d_runs) {
    b->d_runs = balloc(b, sizeof(BatchRun<Real>) * nr);
    if (!b->d_runs) return fail(RELPIC_ENOMEM, "batch: table allocation failed");
  }
  if (!ensure(b, b->d_parts, b->parts_cap, hp.size(), sizeof(BatchPart<Real>)) ||
      !ensure(b, b->d_base, b->base_cap, base.size()) || !ensure(b, b->d_count, b->count_cap, hp.size()))
    return fail(RELPIC_ENOMEM, "batch: table allocation failed");
  if (b->ntot > b->sort_cap) {
    for (unsigned **p : {&b->keys, &b->keys2, &b->idx, &b->idx2}) {
      bfree(b, *p);
      *p = (unsigned *)balloc(b, sizeof(unsigned) * b->ntot);
      if (!*p) return fail(RELPIC_ENOMEM, "batch: sort buffer allocation failed");
    }
    b->sort_cap = b->ntot;
  }
  if (!hp.empty())
    HIP_OK(hipMemcpyAsync(b->d_parts, hp.data(), sizeof(BatchPart<Real>) * hp.size(), hipMemcpyHostToDevice, b->st));
  HIP_OK(hipMemcpyAsync(b->d_base, base.data(), sizeof(long long) * base.size(), hipMemcpyHostToDevice, b->st));
  HIP_OK(hipStreamSynchronize(b->st));
  // sort, choose K per set, mark the species sorted
  if (relpic_status e = sort_all<Real>(b, &hp)) return e;
  b->sorted_at = b->bstep;
  {
    int d = 0;
    for (relpic_sim *s : b->runs)
      for (Species &sp : s->sp) {
        sp.sorted_at = s->step;
        if (sp.n <= 0) {
          sp.dirty = false;
          continue;
        }
        sp.K = hp[d++].K;
        sp.dirty = false;
      }
  }
  // push chunks, grouped by run
  std::vector<BatchChunk> ch;
  {
    int d = 0;
    for (int r = 0; r < nr; ++r) {
      hr[r].chunk0 = (int)ch.size();
      while (d < b->nparts && hp[d].run == r) {
        const long long nb = push_blocks(hp[d].p.n, hp[d].K);
        for (long long c = 0; c < nb; ++c) ch.push_back(BatchChunk{d, (int)c});
        ++d;
      }
      hr[r].nchunk = (int)ch.size() - hr[r].chunk0;
    }
  }
  b->nchunks = (int)ch.size();
  if (!ensure(b, b->d_chunks, b->chunks_cap, ch.size()) || !ensure(b, b->d_chunkbox, b->chunkbox_cap, ch.size()))
    return fail(RELPIC_ENOMEM, "batch: chunk table allocation failed");
  if (!b->d_box) b->d_box = (JBox *)balloc(b, sizeof(JBox) * nr);
  if (!b->err) {
    b->err = (int *)balloc(b, 64);
    if (!b->err) return fail(RELPIC_ENOMEM, "batch: allocation failed");
    HIP_OK(hipMemsetAsync(b->err, 0, 64, b->st));
  }
  if (!b->d_box) return fail(RELPIC_ENOMEM, "batch: allocation failed");
  if (!ch.empty())
    HIP_OK(hipMemcpyAsync(b->d_chunks, ch.data(), sizeof(BatchChunk) * ch.size(), hipMemcpyHostToDevice, b->st));
  HIP_OK(hipMemcpyAsync(b->d_parts, hp.data(), sizeof(BatchPart<Real>) * hp.size(), hipMemcpyHostToDevice, b->st));
  HIP_OK(hipMemcpyAsync(b->d_runs, hr.data(), sizeof(BatchRun<Real>) * nr, hipMemcpyHostToDevice, b->st));
  HIP_OK(hipStreamSynchronize(b->st));
  if (relpic_status e = build_tiles<Real>(b)) return e;
  b->sig = signature(b);
  b->prepared = true;
  return RELPIC_OK;
}

// one step, B^{n-1/2} in slot `par`
template <typename Real>
void enqueue_step(relpic_batch *b, int par, hipStream_t st) {
  const auto *runs = (const BatchRun<Real> *)b->d_runs;
  const int nr = (int)b->runs.size();
  launch_batch_curl_e<Real>(runs, b->d_tiles, b->ntiles, field_grid(b), par, 0, st);
  launch_batch_push<Real>(runs, nr, (const BatchPart<Real> *)b->d_parts, b->d_chunks, b->nchunks, par ^ 1,
                          b->d_chunkbox, b->d_box, b->err, st);
  if (b->any_custom) launch_batch_jcorr<Real>(runs, nr, b->d_box, st);
  launch_batch_curl_b<Real>(runs, b->d_tiles, b->ntiles, field_grid(b), par ^ 1, st);
  launch_batch_add_j<Real>(runs, nr, b->d_box, st);
}

template <typename Real>
relpic_status capture(relpic_batch *b, int par) {
  if (!b->cap_st) HIP_OK(hipStreamCreateWithFlags(&b->cap_st, hipStreamNonBlocking));
  HIP_OK(hipStreamBeginCapture(b->cap_st, hipStreamCaptureModeRelaxed));
  for (int k = 0; k < b->graph_steps; ++k) enqueue_step<Real>(b, par ^ (k & 1), b->cap_st);
  hipGraph_t g = nullptr;
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamEndCapture(b->cap_st, &g);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(RELPIC_EDEVICE, std::string("batch: graph capture failed: ") +
                                    hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  hipGraphExec_t x = nullptr;
  const hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e3 != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(RELPIC_EDEVICE, std::string("batch: graph instantiation failed: ") + hipGetErrorString(e3));
  }
  b->graph[par] = g;
  b->gexec[par] = x;
  return RELPIC_OK;
}

template <typename Real>
relpic_status ensure_prepared(relpic_batch *b) {
  if (b->prepared && slots_match(b) && signature(b) == b->sig) return RELPIC_OK;
  return prepare<Real>(b);
}

template <typename Real>
relpic_status do_batch_steps(relpic_batch *b, long long nsteps) {
  if (relpic_status e = ensure_prepared<Real>(b)) return e;
  if (nsteps == 0) return RELPIC_OK;
  const auto *runs = (const BatchRun<Real> *)b->d_runs;
  // prologue: B^{n-1/2} = B^n + (dt/2) curl+ E^n into the other slot
  launch_batch_curl_e<Real>(runs, b->d_tiles, b->ntiles, field_grid(b), b->canon, 1, b->st);
  int par = 1 - b->canon;
  const int G = b->graph_steps;
  const int sort_every = G > 0 ? G : kSortEvery;
  long long left = nsteps;
  while (left > 0) {
    if (b->bstep % sort_every == 0 && b->sorted_at != b->bstep) {
      if (relpic_status e = sort_all<Real>(b, nullptr)) return e;
      b->sorted_at = b->bstep;
    }
    if (G > 0 && b->bstep % G == 0 && left >= G) {
      if (!b->gexec[par])
        if (relpic_status e = capture<Real>(b, par)) return e;
      HIP_OK(hipGraphLaunch(b->gexec[par], b->st));
      b->bstep += G;
      left -= G;
    } else {
      enqueue_step<Real>(b, par, b->st);
      par ^= 1;
      b->bstep += 1;
      left -= 1;
    }
  }
  // epilogue: B^{n+1} = B^{n+1/2} - (dt/2) curl+ E^{n+1}
  launch_batch_curl_e<Real>(runs, b->d_tiles, b->ntiles, field_grid(b), par, 2, b->st);
  b->canon = 1 - par;
  HIP_OK(hipGetLastError());
  for (size_t r = 0; r < b->runs.size(); ++r) {
    relpic_sim *s = b->runs[r];
    for (int d = 0; d < 3; ++d) {
      s->F[3 + d] = b->slot[b->canon][3 * r + d];
      s->Bx[d] = b->slot[1 - b->canon][3 * r + d];
    }
    s->step += nsteps;
  }
  return RELPIC_OK;
}

// Average time of the B update (curl E, full step) over `reps` launches with
// the current tiling.  It writes only the slot that is free between calls.
template <typename Real>
relpic_status time_curl_e(relpic_batch *b, int reps, double *ms) {
  const auto *runs = (const BatchRun<Real> *)b->d_runs;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  for (int k = 0; k < 2; ++k) launch_batch_curl_e<Real>(runs, b->d_tiles, b->ntiles, field_grid(b), b->canon, 0, b->st);
  (void)hipEventRecord(e0, b->st);
  for (int k = 0; k < reps; ++k)
    launch_batch_curl_e<Real>(runs, b->d_tiles, b->ntiles, field_grid(b), b->canon, 0, b->st);
  (void)hipEventRecord(e1, b->st);
  hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(RELPIC_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
  *ms = (double)t / reps;
  return RELPIC_OK;
}

// Autotuner: time the whole batch with each tile shape on every run, fit a
// cost per tile for each shape from those timings, give every run the shape
// with the lowest modelled cost (its tile count times the shape's cost),
// time that assignment, then try persistent grids for the best assignment.
template <typename Real>
relpic_status do_autotune(relpic_batch *b, int reps, relpic_batch_tune *out) {
  if (relpic_status e = ensure_prepared<Real>(b)) return e;
  const int nr = (int)b->runs.size();
  relpic_batch_tune rep{};
  double per_tile[kNumShapes];
  std::vector<int> best_shape;
  double best = 1e300;
  for (int s = 0; s < kNumShapes; ++s) {
    b->shape.assign(nr, s);
    b->grid_wg = 0;
    if (relpic_status e = build_tiles<Real>(b)) return e;
    double ms;
    if (relpic_status e = time_curl_e<Real>(b, reps, &ms)) return e;
    rep.ms_uniform[s] = ms;
    per_tile[s] = ms / b->ntiles;
    if (ms < best) {
      best = ms;
      best_shape = b->shape;
      rep.choice = s;
    }
  }
  for (int r = 0; r < nr; ++r) {
    int k = 0;
    for (int s = 1; s < kNumShapes; ++s)
      if (shape_tiles(b->runs[r], s) * per_tile[s] < shape_tiles(b->runs[r], k) * per_tile[k]) k = s;
    b->shape[r] = k;
  }
  if (relpic_status e = build_tiles<Real>(b)) return e;
  if (relpic_status e = time_curl_e<Real>(b, reps, &rep.ms_model)) return e;
  if (rep.ms_model < best) {
    best = rep.ms_model;
    best_shape = b->shape;
    rep.choice = kNumShapes;
  }
  b->shape = best_shape;
  if (relpic_status e = build_tiles<Real>(b)) return e;
  int best_grid = 0;
  const int grids[2] = {256 * 16, 256 * 32};
  for (int k = 0; k < 2; ++k) {
    if (grids[k] >= b->ntiles) continue;
    b->grid_wg = grids[k];
    double ms;
    if (relpic_status e = time_curl_e<Real>(b, reps, &ms)) return e;
    rep.ms_persistent[k] = ms;
    if (ms < best) {
      best = ms;
      best_grid = grids[k];
    }
  }
  b->grid_wg = best_grid;
  rep.grid_workgroups = field_grid(b);
  rep.ms_chosen = best;
  for (int s = 0; s < kNumShapes; ++s) rep.runs_per_shape[s] = 0;
  for (int r = 0; r < nr; ++r) rep.runs_per_shape[b->shape[r]] += 1;
  drop_graphs(b);
  if (out) *out = rep;
  return RELPIC_OK;
}

relpic_status check_batch(relpic_batch *b) {
  if (!b) return fail(RELPIC_EINVAL, "null batch handle");
  return RELPIC_OK;
}

void destroy_batch(relpic_batch *b) {
  (void)hipStreamSynchronize(b->st);
  drop_graphs(b);
  if (b->cap_st) (void)hipStreamDestroy(b->cap_st);
  while (!b->owned.empty()) bfree(b, b->owned.back().first);
  for (relpic_sim *s : b->runs) relpic_destroy(s);
  delete b;
}

}  // namespace

extern "C" {

relpic_status relpic_batch_create(int nruns, const relpic_grid *grids, const relpic_solver *solvers,
                                  relpic_precision prec, const relpic_device *dev, relpic_batch **out) {
  return guarded("batch_create", [&]() -> relpic_status {
    if (!out || !grids || nruns < 1 || nruns > (1 << 20)) return fail(RELPIC_EINVAL, "batch_create: bad arguments");
    *out = nullptr;
    for (int r = 0; r < nruns; ++r)
      if (grids[r].ndim != 2 || grids[r].bc1 != RELPIC_BC_PERIODIC)
        return fail(RELPIC_EINVAL, "batch_create: every run must be 2D with a periodic x1 boundary");
    for (int r = 0; solvers && r < nruns; ++r)
      if (solvers[r].MB != 0)
        return fail(RELPIC_EINVAL, "batch_create: batched runs use one axial operator on E and B (MB = 0)");
    relpic_batch *b = new (std::nothrow) relpic_batch();
    if (!b) return fail(RELPIC_ENOMEM, "batch_create: host allocation failed");
    b->prec = prec;
    b->esz = prec == RELPIC_FP32 ? 4 : 8;
    if (dev) b->dev = *dev;
    b->st = (hipStream_t)b->dev.stream;
    for (int r = 0; r < nruns; ++r) {
      relpic_sim *s = nullptr;
      const relpic_status e = relpic_create(&grids[r], solvers ? &solvers[r] : nullptr, prec, dev, &s);
      if (e != RELPIC_OK) {
        const std::string msg = std::string("batch_create: run ") + std::to_string(r) + ": " + relpic_last_error();
        destroy_batch(b);
        return fail(e, msg);
      }
      b->runs.push_back(s);
      b->shape.push_back(kDefaultShape);
    }
    *out = b;
    return RELPIC_OK;
  });
}

relpic_status relpic_batch_destroy(relpic_batch *b) {
  return guarded("batch_destroy", [&]() -> relpic_status {
    if (b) destroy_batch(b);
    return RELPIC_OK;
  });
}

relpic_status relpic_batch_run(relpic_batch *b, int run, relpic_sim **sim) {
  return guarded("batch_run", [&]() -> relpic_status {
    if (relpic_status e = check_batch(b)) return e;
    if (!sim || run < 0 || run >= (int)b->runs.size()) return fail(RELPIC_EINVAL, "batch_run: bad run index");
    *sim = b->runs[run];
    return RELPIC_OK;
  });
}

relpic_status relpic_batch_step(relpic_batch *b, int64_t nsteps) {
  return guarded("batch_step", [&]() -> relpic_status {
    if (relpic_status e = check_batch(b)) return e;
    if (nsteps < 0) return fail(RELPIC_EINVAL, "batch_step: negative count");
    if (b->prec == RELPIC_FP32) return do_batch_steps<float>(b, nsteps);
    return do_batch_steps<double>(b, nsteps);
  });
}

relpic_status relpic_batch_sync(relpic_batch *b) {
  return guarded("batch_sync", [&]() -> relpic_status {
    if (relpic_status e = check_batch(b)) return e;
    HIP_OK(hipStreamSynchronize(b->st));
    if (b->err) {
      int err = 0;
      HIP_OK(hipMemcpy(&err, b->err, sizeof(int), hipMemcpyDeviceToHost));
      if (err) {
        char buf[96];
        std::snprintf(buf, sizeof buf, "batch kernel error word 0x%x (1: moved > 1 cell, 2: NaN momentum)", err);
        return fail(RELPIC_EDEVICE, buf);
      }
    }
    return RELPIC_OK;
  });
}

relpic_status relpic_batch_set_graph_steps(relpic_batch *b, int steps) {
  return guarded("batch_set_graph_steps", [&]() -> relpic_status {
    if (relpic_status e = check_batch(b)) return e;
    if (steps < 0 || (steps & 1) || steps > 100000)
      return fail(RELPIC_EINVAL, "batch_set_graph_steps: steps must be even, 0 .. 100000");
    b->graph_steps = steps;
    drop_graphs(b);
    return RELPIC_OK;
  });
}

relpic_status relpic_batch_set_tiling(relpic_batch *b, const int *shape, int grid_workgroups) {
  return guarded("batch_set_tiling", [&]() -> relpic_status {
    if (relpic_status e = check_batch(b)) return e;
    if (grid_workgroups < 0 || (grid_workgroups % 8) != 0)
      return fail(RELPIC_EINVAL, "batch_set_tiling: grid_workgroups must be a non-negative multiple of 8");
    if (shape)
      for (size_t r = 0; r < b->runs.size(); ++r)
        if (shape[r] < 0 || shape[r] >= kNumShapes) return fail(RELPIC_EINVAL, "batch_set_tiling: bad shape");
    if (shape) b->shape.assign(shape, shape + b->runs.size());
    b->grid_wg = grid_workgroups;
    if (!b->prepared) return RELPIC_OK;
    return b->prec == RELPIC_FP32 ? build_tiles<float>(b) : build_tiles<double>(b);
  });
}

relpic_status relpic_batch_get_tiling(relpic_batch *b, int *shape, int *grid_workgroups) {
  return guarded("batch_get_tiling", [&]() -> relpic_status {
    if (relpic_status e = check_batch(b)) return e;
    if (shape) std::copy(b->shape.begin(), b->shape.end(), shape);
    if (grid_workgroups) *grid_workgroups = b->grid_wg;
    return RELPIC_OK;
  });
}

relpic_status relpic_batch_autotune(relpic_batch *b, int reps, relpic_batch_tune *out) {
  return guarded("batch_autotune", [&]() -> relpic_status {
    if (relpic_status e = check_batch(b)) return e;
    if (reps < 1 || reps > 10000) return fail(RELPIC_EINVAL, "batch_autotune: reps must be in 1..10000");
    return b->prec == RELPIC_FP32 ? do_autotune<float>(b, reps, out) : do_autotune<double>(b, reps, out);
  });
}

relpic_status relpic_batch_read_field(relpic_batch *b, int run, relpic_field f, double *host, int64_t count) {
  return guarded("batch_read_field", [&]() -> relpic_status {
    if (relpic_status e = check_batch(b)) return e;
    if (run < 0 || run >= (int)b->runs.size()) return fail(RELPIC_EINVAL, "batch_read_field: bad run index");
    return relpic_read_field(b->runs[run], f, host, count);
  });
}

}  // extern "C"
