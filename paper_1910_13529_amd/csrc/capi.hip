// C ABI and host engine of relpic: owns the device arrays of one simulation,
// validates descriptors, and enqueues the per-step kernel sequence on the
// caller's stream:
//   push+deposit (per species) -> [J1 correction] -> B half -> E -> B half
//   -> [window shift: zero the new leading slab, inject plasma]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "engine.h"
#include "solver_setup.h"

using namespace relpic;

namespace relpic_host {

namespace {
// the last failure's message on this thread (fixed storage: setting it never allocates)
thread_local char g_last_error[512] = "";

void set_last_error(const char *a, const char *b) noexcept {
  size_t k = 0;
  for (const char *p = a; p && *p && k + 1 < sizeof g_last_error; ++p) g_last_error[k++] = *p;
  if (b) {
    for (const char *p = ": "; *p && k + 1 < sizeof g_last_error; ++p) g_last_error[k++] = *p;
    for (const char *p = b; *p && k + 1 < sizeof g_last_error; ++p) g_last_error[k++] = *p;
  }
  g_last_error[k] = 0;
}
}  // namespace

relpic_status fail(relpic_status s, const std::string &msg) {
  set_last_error(msg.c_str(), nullptr);
  return s;
}

relpic_status fail_noalloc(relpic_status s, const char *where, const char *what) noexcept {
  set_last_error(where, what);
  return s;
}

const char *last_error() { return g_last_error; }

void *dev_alloc(relpic_sim *s, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void *p = nullptr;
  if (s->dev.alloc) {
    p = s->dev.alloc(bytes, s->dev.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) s->owned.push_back(p);
  return p;
}

// free one allocation made by dev_alloc (scratch of a set-up call)
void dev_release(relpic_sim *s, void *p) {
  if (!p) return;
  for (size_t i = 0; i < s->owned.size(); ++i)
    if (s->owned[i] == p) {
      if (s->dev.free)
        s->dev.free(p, s->dev.user);
      else if (!s->dev.alloc)
        (void)hipFree(p);
      s->owned.erase(s->owned.begin() + (long)i);
      return;
    }
}

void dev_free_all(relpic_sim *s) {
  for (void *p : s->owned) {
    if (s->dev.free)
      s->dev.free(p, s->dev.user);
    else if (!s->dev.alloc)
      (void)hipFree(p);
  }
  s->owned.clear();
}

}  // namespace relpic_host

using namespace relpic_host;

namespace {

// Bracket one launch with events when profiling is on.
struct ProfScope {
  relpic_sim *s;
  int cls;
  size_t idx = 0;
  bool on = false;
  ProfScope(relpic_sim *s_, int c) : s(s_), cls(c) {
    if (!s->prof) return;
    while (s->ev_pool.size() < s->ev_used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      s->ev_pool.push_back(e);
    }
    idx = s->ev_used;
    s->ev_used += 2;
    on = hipEventRecord(s->ev_pool[idx], s->st) == hipSuccess;
  }
  ~ProfScope() {
    if (!on) return;
    if (hipEventRecord(s->ev_pool[idx + 1], s->st) == hipSuccess) s->ev_marks.emplace_back(cls, idx);
  }
};

long long window_target(const relpic_sim *s, long long steps_done) {
  return (long long)std::floor((double)steps_done * s->grid.window_speed * s->grid.dt / s->dx[0] + 1e-9);
}


// Key order by density: a sparse species (a plasma filling the grid) sorts
// by 3D tiles so that a push chunk covers a compact box; a dense bunch, whose
// chunks sit in one or two cells either way, keeps plain row order (its
// chunks then straddle no tile seams).  Mean particles per occupied cell
// below kTileBelow switches to tiles, above kRowsAbove back to rows.
constexpr double kTileBelow = 64.0, kRowsAbove = 128.0;
// particles per occupied cell from which a tile-sorted FP32 species pushes
// without the wavefront rounds (runs of 6 and more fill most of a cell group)
constexpr double kLongRunsPpc = 6.0;
// largest key space sorted by counting (4 bytes per bucket)
constexpr long long kCountingSortMaxKeys = 1LL << 28;
constexpr long long kMinPushChunks = 512;

// Sort a species by cell (dropped particles last), drop the dropped ones,
// and pick the push chunk size from the particles per occupied cell.  When
// the measured density asks for the other key order, sort once more in it.
template <typename Real>
relpic_status do_sort(relpic_sim *s, Species &sp) {
  sp.dirty = false;
  sp.sorted_at = s->step;
  sp.ntiles = sp.n_tiled = 0;
  sp.long_runs = false;
  if (sp.n <= 1) return RELPIC_OK;
  Particles<Real> src = parts<Real>(sp);
  const Geo g = make_geo(s);
  const bool tiles = sp.tile_keys && sort_tiles_fit(g);
  // tile x1 width 2^tx: FP64 tiles are half as wide (LDS holds half the cells)
  const int tx = sizeof(Real) == 8 ? 2 : 3;
  launch_sort_keys<Real>(g, src, tiles ? tx : 0, sp.keys, sp.idx, s->st);
  unsigned long long *cnt = (unsigned long long *)(s->dbuf + 6);
  unsigned long long *runs = (unsigned long long *)(s->dbuf + 7);
  HIP_OK(hipMemsetAsync(s->dbuf + 6, 0, 2 * sizeof(double), s->st));
  // key space: the cells in tile order, or the packed cell index
  long long nkeys = g.N;
  if (tiles) {
    const long long nt1 = (g.n1 + (1 << tx) - 1) >> tx, nt2 = (g.n2 + 3) / 4, nt3 = g.n3 > 1 ? (g.n3 + 3) / 4 : 1;
    nkeys = nt1 * nt2 * nt3 * ((long long)(g.n3 > 1 ? 16 : 4) << tx);
  }
  // counting sort (hand-written, two passes over the keys) for a species in
  // tile order (a few particles per cell: short runs spread over the
  // buckets) when the buckets fit; radix sort otherwise (a dense bunch's
  // thousands of particles per cell turn the bucket atomics into
  // same-address chains: 1.4-4.5 ms per pass on the 3D beam against 0.3 ms
  // for the whole radix sort)
  const bool counting = tiles && nkeys <= kCountingSortMaxKeys;
  if (counting) {
    const long long nb = key_scan_blocks((unsigned)nkeys);
    if (nkeys > s->kcount_cap) {
      s->kcount = (unsigned *)dev_alloc(s, sizeof(unsigned) * (size_t)nkeys);
      if (!s->kcount) return fail(RELPIC_ENOMEM, "sort: bucket allocation failed");
      s->kcount_cap = nkeys;
    }
    if (nb > s->kblocks_cap) {
      s->kbsum = (unsigned long long *)dev_alloc(s, sizeof(unsigned long long) * (size_t)nb);
      s->kbocc = (unsigned *)dev_alloc(s, sizeof(unsigned) * (size_t)nb);
      if (!s->kbsum || !s->kbocc) return fail(RELPIC_ENOMEM, "sort: scan scratch allocation failed");
      s->kblocks_cap = nb;
    }
    HIP_OK(hipMemsetAsync(s->kcount, 0, sizeof(unsigned) * (size_t)nkeys, s->st));
    launch_key_sort(sp.keys, sp.n, (unsigned)nkeys, s->kcount, s->kbsum, s->kbocc, cnt, sp.keys2, sp.idx2, s->st);
  } else {
    size_t need = 0;
    HIP_OK(sort_pairs(nullptr, need, sp.keys, sp.keys2, sp.idx, sp.idx2, sp.n, s->st));
    if (need > sp.sort_tmp_bytes) {
      sp.sort_tmp = dev_alloc(s, need);
      if (!sp.sort_tmp) return fail(RELPIC_ENOMEM, "sort: temporary storage allocation failed");
      sp.sort_tmp_bytes = need;
    }
    HIP_OK(sort_pairs(sp.sort_tmp, need, sp.keys, sp.keys2, sp.idx, sp.idx2, sp.n, s->st));
  }
  Particles<Real> dst = src;
  dst.cell = sp.cell2;
  dst.o1 = (Real *)sp.o2[0];
  dst.o2 = (Real *)sp.o2[1];
  dst.o3 = (Real *)sp.o2[2];
  dst.u1 = (Real *)sp.u2[0];
  dst.u2 = (Real *)sp.u2[1];
  dst.u3 = (Real *)sp.u2[2];
  // the counting sort leaves the alive count in cnt[0] and the distinct
  // cells in cnt[1]; the radix sort keeps the dropped particles (last)
  launch_permute<Real>(src, dst, sp.id, sp.id2, sp.idx2, s->ndim, s->st, counting ? cnt : nullptr);
  if (!counting) launch_count_runs(sp.keys2, sp.n, runs, cnt, s->st);
  unsigned long long h[2] = {0, 0};
  HIP_OK(hipMemcpyAsync(h, s->dbuf + 6, sizeof(h), hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  std::swap(sp.cell, sp.cell2);
  for (int d = 0; d < 3; ++d) {
    std::swap(sp.o[d], sp.o2[d]);
    std::swap(sp.u[d], sp.u2[d]);
  }
  std::swap(sp.id, sp.id2);
  sp.n = (long long)h[0];
  const double ppc = h[1] ? (double)h[0] / (double)h[1] : 0.0;
  const bool want = sort_tiles_fit(g) && sp.n > 1 && ppc < (sp.tile_keys ? kRowsAbove : kTileBelow);
  if (want != tiles) {
    sp.tile_keys = want;
    return do_sort<Real>(s, sp);
  }
  sp.ntiles = sp.n_tiled = 0;
  // cells holding runs of several particles (a plasma at a few per cell):
  // the cell groups take nearly every lane, the rest deposit directly
  sp.long_runs = tiles && ppc >= kLongRunsPpc;
  if (tiles) {
    // chunks of 256 K particles.  2D: at most one tile's worth, so a chunk
    // spans parts of at most two x1-neighbouring tiles, whose cells with the
    // deposit halo fit the push's LDS tile.  3D (the sorted particles go one
    // sort tile per workgroup below): chunks for the particles appended after
    // this sort, at most one injected transverse block's worth, whose one x1
    // cell with the halo (5 x 12 x 12 cells) fits the LDS tile with the
    // current in FP64 words; a 1024-particle chunk of an 8-per-cell slab
    // (5 x 12 x 20) does not
    const double per_chunk =
        s->ndim == 3 ? ppc * (double)(kInjBlock * kInjBlock) : ppc * (double)(4 << tx);
    sp.K = per_chunk >= 2048.0 ? 8 : (per_chunk >= 1024.0 ? 4 : (per_chunk >= 512.0 ? 2 : 1));
    // the sorted particles are pushed one sort tile per workgroup: the
    // chunk's cells are exactly one tile (plus the particles' drift since)
    if (s->ndim == 3 && sp.n > 0) {
      const long long nt1 = (g.n1 + (1 << tx) - 1) >> tx, nt2 = (g.n2 + 3) / 4, nt3 = (g.n3 + 3) / 4;
      const long long ntiles = nt1 * nt2 * nt3;
      if (ntiles > sp.tiles_cap) {
        sp.tile_first = (int *)dev_alloc(s, sizeof(int) * (size_t)ntiles);
        sp.tile_end = (int *)dev_alloc(s, sizeof(int) * (size_t)ntiles);
        if (!sp.tile_first || !sp.tile_end) return fail(RELPIC_ENOMEM, "sort: tile range allocation failed");
        sp.tiles_cap = ntiles;
      }
      HIP_OK(hipMemsetAsync(sp.tile_first, 0, sizeof(int) * (size_t)ntiles, s->st));
      HIP_OK(hipMemsetAsync(sp.tile_end, 0, sizeof(int) * (size_t)ntiles, s->st));
      launch_tile_ranges(sp.keys2, sp.n, 4 + tx, ntiles, sp.tile_first, sp.tile_end, s->st);
      sp.ntiles = ntiles;
      sp.n_tiled = sp.n;
    }
  } else {
    // row order: 1024-particle chunks at most (2048 measured 6% slower on a
    // dense bunch, 512 2% slower)
    sp.K = ppc >= 64.0 ? 4 : (ppc >= 16.0 ? 2 : 1);
  }
  // a small species still gets about two chunks per CU (a dense bunch of
  // 65536 particles in 32 chunks left seven of eight CUs idle)
  while (sp.K > 1 && push_blocks(sp.n, sp.K) < kMinPushChunks) sp.K /= 2;
  return RELPIC_OK;
}


// Bout = Bin - c curl+ E (c = dt for a full step, +-dt/2 for half steps)
template <typename Real>
void curl_e(relpic_sim *s, const Geo &g, Real *const Bin[3], Real *const Bout[3], double c) {
  const Fields<Real> f = fields<Real>(s);
  const Real h2 = (Real)(c / s->dx[1]), h3 = (Real)(s->ndim == 3 ? c / s->dx[2] : 0.0);
  launch_curl_e<Real>(s->ndim, g, f, Bin, Bout, axial_scaled<Real>(s, c), h2, h3, s->st);
}

// x1 widening of the deposit box that holds the current the E update adds:
// the J1 correction's half-width and the filter's reach
int current_pad(const relpic_sim *s) {
  return (s->correct ? s->ng : 0) + (s->filt_npass > 0 ? s->filt_npass + 1 : 0);
}

template <typename Real>
relpic_status do_steps(relpic_sim *s, long long nsteps) {
  if (nsteps == 0) return RELPIC_OK;
  const double dt = s->grid.dt;
  const Axial<Real> axE = axial_scaled_b<Real>(s, dt);  // E update: the operator on B
  const Real e2 = (Real)(dt / s->dx[1]), e3 = (Real)(s->ndim == 3 ? dt / s->dx[2] : 0.0);
  const bool window = s->grid.bc1 == RELPIC_BC_WINDOW;
  Real *Ba[3] = {(Real *)s->F[3], (Real *)s->F[4], (Real *)s->F[5]};
  Real *Bb[3] = {(Real *)s->Bx[0], (Real *)s->Bx[1], (Real *)s->Bx[2]};
  auto swapB = [&]() {
    for (int d = 0; d < 3; ++d) std::swap(Ba[d], Bb[d]);
  };
  // prologue: B^{n-1/2} = B^n + (dt/2) curl+ E^n
  {
    ProfScope ps(s, 2);
    curl_e<Real>(s, make_geo(s), Ba, Bb, -0.5 * dt);
  }
  swapB();
  relpic_status status = RELPIC_OK;
  // With the fused update, the step's E update also produces the next B:
  // b_ahead = B^{n+1/2} of the coming step is already in Bb, b_final = the
  // last step produced B^{n+1} (the epilogue) itself.
  bool b_ahead = false, b_final = false;
  for (long long it = 0; it < nsteps; ++it) {
    for (auto &sp : s->sp)
      if (sp.dirty || (s->sort_interval > 0 && s->step - sp.sorted_at >= s->sort_interval))
        if ((status = do_sort<Real>(s, sp))) break;
    if (status) break;
    int shift = 0;
    if (window) {
      const long long tgt = window_target(s, s->step + 1);
      if (tgt - s->ws > 1) {
        status = fail(RELPIC_EUNSTABLE, "window moves more than one cell per step");
        break;
      }
      shift = tgt > s->ws ? 1 : 0;
    }
    const Geo g = make_geo(s);
    JBox *box = s->jbox + (s->step & 1);
    JBox *next = s->jbox + ((s->step + 1) & 1);
    // B^{n+1/2} = B^{n-1/2} - dt curl+ E^n
    if (!b_ahead) {
      ProfScope ps(s, 2);
      curl_e<Real>(s, g, Ba, Bb, dt);
    }
    b_ahead = false;
    Fields<Real> f = fields<Real>(s);
    f.B1 = Ba[0];
    f.B2 = Ba[1];
    f.B3 = Ba[2];
    const HalfB<Real> Bh{Bb[0], Bb[1], Bb[2]};
    for (size_t si = 0; si < s->sp.size(); ++si) {
      Species &sp = s->sp[si];
      const PushParams<Real> q = push_params<Real>(s, sp, shift);
      PushChunks pc;
      pc.first = sp.tile_first;
      pc.end = sp.tile_end;
      pc.ntiles = sp.ntiles;
      pc.nsorted = sp.n_tiled;
      pc.K = sp.K;
      const long long nb = push_grid(pc, sp.n);
      if (nb > s->blockbox_n) {
        s->blockbox = (JBox *)dev_alloc(s, sizeof(JBox) * (size_t)nb);
        if (!s->blockbox) {
          status = fail(RELPIC_ENOMEM, "step: allocation of workgroup boxes failed");
          break;
        }
        s->blockbox_n = nb;
      }
      {
        ProfScope ps(s, 0 + 64 * (int)(si + 1));
        launch_push_deposit<Real>(s->ndim, g, f, Bh, parts<Real>(sp), q, pc, sp.tile_keys, sp.long_runs, s->blockbox,
                                  s->err, s->st);
      }
      ProfScope ps(s, 6);
      launch_merge_boxes(s->blockbox, nb, box, s->st);
    }
    if (status) break;
    const Real *J1src = f.J1;
    if (s->correct) {
      ProfScope ps(s, 1);
      launch_jcorr<Real>(g, f.J1, f.J1c, (const Real *)s->taps, s->ng, box, s->st);
      J1src = f.J1c;
    }
    if (s->filt_npass > 0) {
      // after the correction, on the current the E update takes
      ProfScope ps(s, 8);
      launch_filter_rows<Real>(g, const_cast<Real *>(J1src), f.J2, f.J3, box, s->correct ? s->ng : 0, s->filt_npass,
                               (Real)(-0.25 * s->filt_comp), (Real)(1.0 + 0.5 * s->filt_comp), s->st);
    }
    const int jpad = current_pad(s);
    // E^{n+1} = E^n + dt (curl- B^{n+1/2} - J^{n+1/2})
    f.B1 = Bb[0];
    f.B2 = Bb[1];
    f.B3 = Bb[2];
    if (s->fuse) {
      // fused: also B^{n+3/2} (or B^{n+1} after the last step) into Ba,
      // which held B^{n-1/2}; E^{n+1} into the second E buffer; a window
      // shift after it is applied to the result (launch_shift_fused)
      const bool last = it + 1 == nsteps;
      const double fb = last ? 0.5 * dt : dt;
      Real *Ein[3] = {f.E1, f.E2, f.E3};
      Real *Eout[3] = {(Real *)s->Ex[0], (Real *)s->Ex[1], (Real *)s->Ex[2]};
      {
        ProfScope ps(s, 7);
        launch_leap<Real>(g, Ein, Eout, Bb, Ba, J1src, f.J2, f.J3, box, jpad, (Real)dt, axE, e2, e3,
                          axial_scaled<Real>(s, fb), (Real)(fb / s->dx[1]), (Real)(fb / s->dx[2]), s->st);
      }
      {
        ProfScope ps(s, 5);
        launch_clear_j<Real>(g, f, box, jpad, next, s->st);
      }
      for (int d = 0; d < 3; ++d) std::swap(s->F[d], s->Ex[d]);
      b_ahead = !last;
      b_final = last;
    } else {
      {
        ProfScope ps(s, 3);
        launch_curl_b<Real>(s->ndim, g, f, axE, e2, e3, s->st);
      }
      {
        ProfScope ps(s, 5);
        launch_add_j<Real>(g, f, J1src, (Real)dt, box, jpad, next, s->st);
      }
    }
    swapB();
    s->step += 1;
    if (shift) {
      ProfScope ps(s, 4);
      Fields<Real> fz = fields<Real>(s);
      if (s->fuse) {
        // Ba: B^{n+1/2}, Bb: the B the fused update produced
        Real *E[3] = {fz.E1, fz.E2, fz.E3};
        launch_shift_fused<Real>(g, E, Ba, Bb, g.ws_mod, axial_scaled<Real>(s, 0.5 * dt), (Real)(b_final ? 0.0 : 1.0),
                                 s->st);
      } else {
        fz.B1 = Ba[0];
        fz.B2 = Ba[1];
        fz.B3 = Ba[2];
        launch_new_slab<Real>(g, fz, Bb, g.ws_mod, axial_scaled<Real>(s, 0.5 * dt), s->st);
      }
      s->ws += 1;
      const Geo g2 = make_geo(s);
      for (auto &sp : s->sp) {
        if (!sp.inject) continue;
        const long long nnew = (long long)sp.ppc[0] * sp.ppc[1] * sp.ppc[2] * s->n[1] * s->n[2];
        if (sp.n + nnew > sp.cap) {
          status = fail(RELPIC_ERANGE, "injection exceeds species capacity");
          break;
        }
        launch_inject_slab<Real>(s->ndim, g2, parts<Real>(sp), sp.id, sp.n, s->n[0] - 3, sp.ppc[0], sp.ppc[1],
                                 sp.ppc[2], sp.uth, sp.seed, sp.inj_count, sp.next_id, s->st);
        sp.n += nnew;
        sp.next_id += nnew;
        sp.inj_count += (unsigned long long)nnew;
      }
      if (status) break;
    }
  }
  // epilogue: B^{n+1} = B^{n+1/2} - (dt/2) curl+ E^{n+1}, back in the canonical buffer
  if (!b_final) {
    ProfScope ps(s, 2);
    curl_e<Real>(s, make_geo(s), Ba, Bb, 0.5 * dt);
  }
  swapB();
  for (int d = 0; d < 3; ++d) {
    s->F[3 + d] = Ba[d];
    s->Bx[d] = Bb[d];
  }
  if (status) return status;
  HIP_OK(hipGetLastError());
  return RELPIC_OK;
}

template <typename Real>
relpic_status do_diag(relpic_sim *s, relpic_diag *out) {
  const Geo g = make_geo(s);
  Fields<Real> f = fields<Real>(s);
  HIP_OK(hipMemsetAsync(s->dbuf, 0, 8 * sizeof(double), s->st));
  HIP_OK(hipMemsetAsync(s->rho, 0, sizeof(double) * s->N, s->st));
  launch_diag_field_energy<Real>(g, f, s->dbuf + 0, s->st);
  const double dV = cell_volume(s);
  for (auto &sp : s->sp) {
    // a ballistic species (q/m = 0) has no mass in the model: its kinetic energy is not counted
    launch_diag_kinetic<Real>(parts<Real>(sp), sp.qm != 0.0 ? sp.Q / sp.qm : 0.0, s->dbuf + 1,
                              (unsigned long long *)(s->dbuf + 5), s->st);
    launch_diag_rho<Real>(s->ndim, g, parts<Real>(sp), sp.Q / dV, s->rho, s->st);
  }
  if (s->filt_npass > 0)  // Gauss's law holds for the filtered density
    launch_filter_rows<double>(g, s->rho, nullptr, nullptr, nullptr, 0, s->filt_npass, -0.25 * s->filt_comp,
                               1.0 + 0.5 * s->filt_comp, s->st);
  Axial<double> c1{};
  c1.M = s->M;
  for (int l = 0; l < s->M; ++l) c1.c[l] = s->CB[l] / s->dx[0];  // Gauss: the operator on B
  launch_diag_gauss<Real>(s->ndim, g, f, c1, 1.0 / s->dx[1], s->ndim == 3 ? 1.0 / s->dx[2] : 0.0, s->rho, s->rho_bg,
                          2 * s->M + 2, s->dbuf + 2, s->st);
  double h[8];
  int err = 0;
  HIP_OK(hipMemcpyAsync(h, s->dbuf, sizeof(h), hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipMemcpyAsync(&err, s->err, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIP_OK(hipStreamSynchronize(s->st));
  unsigned long long cnt;
  std::memcpy(&cnt, &h[5], sizeof(cnt));
  out->step = s->step;
  out->window_start = s->ws;
  out->n_alive = (int64_t)cnt;
  out->time = s->step * s->grid.dt;
  out->w_field = h[0] * cell_volume(s);
  out->w_kin = h[1];
  out->gauss_max = h[2];
  out->rho_max = h[3];
  out->charge = h[4] * cell_volume(s);
  out->error_word = err;
  return RELPIC_OK;
}

// host staging buffers hold at most this many elements per array
constexpr long long kStage = 1LL << 22;

// Copy rows [r0, r0 + nr) of a field between its storage order (x1 columns
// rotated by the ring buffer) and a dense FP64 window-relative host array,
// through a bounded staging buffer.
relpic_status copy_rows(relpic_sim *s, int f, double *host, bool to_host) {
  const int n1 = s->n[0];
  const long long rows = s->N / n1;
  const long long per = std::max<long long>(1, kStage / n1);
  const int wsm = make_geo(s).ws_mod;
  std::vector<unsigned char> raw((size_t)std::min(rows, per) * n1 * s->esz);
  for (long long r0 = 0; r0 < rows; r0 += per) {
    const long long nr = std::min(per, rows - r0);
    char *dev = (char *)s->F[f] + (size_t)r0 * n1 * s->esz;
    if (to_host) {
      HIP_OK(hipMemcpyAsync(raw.data(), dev, (size_t)nr * n1 * s->esz, hipMemcpyDeviceToHost, s->st));
      HIP_OK(hipStreamSynchronize(s->st));
    }
    for (long long r = 0; r < nr; ++r)
      for (int l = 0; l < n1; ++l) {
        const long long sidx = r * n1 + (l + wsm) % n1;
        double &h = host[(r0 + r) * n1 + l];
        if (s->esz == 4) {
          float x;
          if (to_host) {
            std::memcpy(&x, &raw[sidx * 4], 4);
            h = x;
          } else {
            x = (float)h;
            std::memcpy(&raw[sidx * 4], &x, 4);
          }
        } else if (to_host) {
          std::memcpy(&h, &raw[sidx * 8], 8);
        } else {
          std::memcpy(&raw[sidx * 8], &h, 8);
        }
      }
    if (!to_host) {
      HIP_OK(hipMemcpyAsync(dev, raw.data(), (size_t)nr * n1 * s->esz, hipMemcpyHostToDevice, s->st));
      HIP_OK(hipStreamSynchronize(s->st));
    }
  }
  return RELPIC_OK;
}

relpic_status check_sim(relpic_sim *s) {
  if (!s) return fail(RELPIC_EINVAL, "null simulation handle");
  return RELPIC_OK;
}

}  // namespace

extern "C" {

const char *relpic_last_error(void) { return last_error(); }

relpic_status relpic_fit_operator(double kappa, int M, int p, double wk1, double nsg, int target, double *C_out,
                                  double *max_rel_err_out) {
  return guarded("fit_operator", [&]() -> relpic_status {
    if (!C_out || M < 1 || M > kMaxM || (target != RELPIC_FIT_TIME && target != RELPIC_FIT_E_WITH_YEE_B))
      return fail(RELPIC_EINVAL, "fit: bad M, target or output pointer");
    std::vector<double> C;
    if (!fit_axial_coefficients(kappa, M, p, wk1, nsg, 2048, C, target))
      return fail(RELPIC_EINVAL, "fit: singular or bad parameters");
    std::copy(C.begin(), C.end(), C_out);
    if (max_rel_err_out) {
      double worst = 0.0;
      for (int q = 1; q <= 2000; ++q) {
        const double kh = 1.0 * q / 2000;
        double v = 0.0;
        for (int l = 1; l <= M; ++l) v += C[l - 1] * std::sin((2 * l - 1) * kh);
        double t = kappa * std::sin(kh / kappa);
        if (target == RELPIC_FIT_E_WITH_YEE_B) t = t * t / std::sin(kh);
        worst = std::max(worst, std::fabs(v - t) / t);
      }
      *max_rel_err_out = worst;
    }
    return RELPIC_OK;
  });
}

relpic_status relpic_fit_coefficients(double kappa, int M, int p, double wk1, double nsg, double *C_out,
                                      double *max_rel_err_out) {
  return guarded("fit_coefficients", [&]() -> relpic_status {
    return relpic_fit_operator(kappa, M, p, wk1, nsg, RELPIC_FIT_TIME, C_out, max_rel_err_out);
  });
}

relpic_status relpic_create(const relpic_grid *grid, const relpic_solver *solver, relpic_precision prec,
                            const relpic_device *dev, relpic_sim **out) {
  return guarded("create", [&]() -> relpic_status {
    if (!grid || !out) return fail(RELPIC_EINVAL, "create: null descriptor");
    *out = nullptr;
    if (grid->ndim != 2 && grid->ndim != 3) return fail(RELPIC_EINVAL, "create: ndim must be 2 or 3");
    if (prec != RELPIC_FP32 && prec != RELPIC_FP64) return fail(RELPIC_EINVAL, "create: bad precision");
    if (grid->bc1 != RELPIC_BC_PERIODIC && grid->bc1 != RELPIC_BC_WINDOW) return fail(RELPIC_EINVAL, "create: bad bc1");
    if (!(grid->dt > 0.0)) return fail(RELPIC_EINVAL, "create: dt must be positive");
    long long N = 1;
    for (int d = 0; d < grid->ndim; ++d) {
      if (grid->n[d] < 1 || grid->n[d] > (1 << 24) || !(grid->dx[d] > 0.0))
        return fail(RELPIC_EINVAL, "create: bad n or dx");
      N *= grid->n[d];
    }
    // kernels address field arrays with 32-bit byte offsets
    if (N * (prec == RELPIC_FP64 ? 8LL : 4LL) >= (1LL << 32))
      return fail(RELPIC_EINVAL, "create: field arrays above 4 GiB each (2^30 cells FP32, 2^29 FP64)");
    if (grid->n[0] < 8 || grid->n[1] < 2 || (grid->ndim == 3 && grid->n[2] < 2))
      return fail(RELPIC_EINVAL, "create: grid too small (n1 >= 8, n2, n3 >= 2)");
    if (grid->n[1] > 65535 || (grid->ndim == 3 && grid->n[2] > 65535))
      return fail(RELPIC_EINVAL, "create: n2 and n3 are limited to 65535 (launch grid rows)");
    // operator on E (d+): M, C; operator on B (d-): MB, CB (MB = 0: the same as on E)
    int ME = 1, MB = 0;
    double CE[kMaxM] = {1.0}, CBv[kMaxM] = {1.0};
    if (solver && solver->M > 1) {
      if (solver->M > kMaxM || !solver->C) return fail(RELPIC_EINVAL, "create: bad solver coefficients");
      ME = solver->M;
      for (int l = 0; l < ME; ++l) CE[l] = solver->C[l];
    } else if (solver && solver->M == 1 && solver->C) {
      CE[0] = solver->C[0];
    }
    if (solver && solver->MB > 0) {
      if (solver->MB > kMaxM || (solver->MB > 1 && !solver->CB))
        return fail(RELPIC_EINVAL, "create: bad coefficients of the operator on B");
      MB = solver->MB;
      for (int l = 0; l < MB; ++l) CBv[l] = solver->CB ? solver->CB[l] : 1.0;
    } else if (solver && solver->MB < 0) {
      return fail(RELPIC_EINVAL, "create: MB must be >= 0");
    }
    // both on M = max(ME, MB) coefficients, the shorter zero-padded
    const int M = std::max(ME, MB);
    double C[kMaxM] = {0.0}, CB[kMaxM] = {0.0};
    for (int l = 0; l < M; ++l) {
      C[l] = l < ME ? CE[l] : 0.0;
      CB[l] = MB == 0 ? C[l] : (l < MB ? CBv[l] : 0.0);
    }
    int MBeff = 1;  // d- stencil width without trailing zeros: wider than two points needs the J1 correction
    for (int l = 0; l < M; ++l)
      if (CB[l] != 0.0) MBeff = l + 1;
    if (2 * M > grid->n[0]) return fail(RELPIC_EINVAL, "create: stencil wider than the grid");
    if (grid->bc1 == RELPIC_BC_WINDOW) {
      if (!(grid->window_speed > 0.0) || grid->window_speed * grid->dt >= grid->dx[0])
        return fail(RELPIC_EINVAL, "create: window must advance less than one cell per step");
    }
    const double cn = courant_number2(grid->ndim, grid->dx, grid->dt, C, CB, M);
    if (!(cn < 1.0)) {
      char buf[128];
      std::snprintf(buf, sizeof buf, "create: Courant number %.6f >= 1", cn);
      return fail(RELPIC_EUNSTABLE, buf);
    }
    // every particle moves less than one cell per step only if dt < dx_d
    for (int d = 0; d < grid->ndim; ++d)
      if (!(grid->dt < grid->dx[d])) return fail(RELPIC_EUNSTABLE, "create: dt must be below every dx");

    relpic_sim *s = new (std::nothrow) relpic_sim();
    if (!s) return fail(RELPIC_ENOMEM, "create: host allocation failed");
    s->grid = *grid;
    s->ndim = grid->ndim;
    for (int d = 0; d < 3; ++d) {
      s->n[d] = d < grid->ndim ? (int)grid->n[d] : 1;
      s->dx[d] = d < grid->ndim ? grid->dx[d] : 1.0;
    }
    s->N = N;
    s->prec = prec;
    s->esz = prec == RELPIC_FP32 ? 4 : 8;
    s->M = M;
    for (int l = 0; l < M; ++l) {
      s->C[l] = C[l];
      s->CB[l] = CB[l];
    }
    s->correct = MBeff > 1;
    if (dev) s->dev = *dev;
    s->st = (hipStream_t)s->dev.stream;
    if (hipSetDevice(s->dev.device) != hipSuccess) {
      delete s;
      return fail(RELPIC_EDEVICE, "create: hipSetDevice failed");
    }
    // the identity (one tap, 1) where no correction is needed, so a kernel that
    // applies the taps anyway leaves J1 unchanged
    std::vector<double> taps(1, 1.0);
    if (s->correct) {
      const double tol = prec == RELPIC_FP64 ? 1e-16 : 1e-9;
      if (!correction_taps(CB, M, tol, kMaxTaps, taps)) {
        delete s;
        return fail(RELPIC_EINVAL, "create: J1 correction does not converge within the tap limit");
      }
      s->ng = (int)taps.size() - 1;
    }
    for (int k = 0; k < 10; ++k) {
      if (k == 9 && M == 1) continue;
      s->F[k] = dev_alloc(s, s->esz * N);
      if (!s->F[k]) {
        dev_free_all(s);
        delete s;
        return fail(RELPIC_ENOMEM, "create: field allocation failed");
      }
    }
    for (int d = 0; d < 3; ++d) {
      s->Bx[d] = dev_alloc(s, s->esz * N);
      if (!s->Bx[d]) {
        dev_free_all(s);
        delete s;
        return fail(RELPIC_ENOMEM, "create: field allocation failed");
      }
    }
    // second E buffer for the fused update, where the grid qualifies (the
    // separate updates remain if it cannot be allocated)
    if (grid->ndim == 3 && (prec == RELPIC_FP32 ? leap_supported<float>(make_geo(s), M)
                                                : leap_supported<double>(make_geo(s), M))) {
      bool ok = true;
      for (int d = 0; d < 3 && ok; ++d) ok = (s->Ex[d] = dev_alloc(s, s->esz * N)) != nullptr;
      s->fuse = ok;
      if (!ok)
        for (int d = 0; d < 3; ++d) s->Ex[d] = nullptr;
    }
    s->jbox = (JBox *)dev_alloc(s, 2 * sizeof(JBox));
    s->err = (int *)dev_alloc(s, 64);
    s->dbuf = (double *)dev_alloc(s, 8 * sizeof(double));
    s->rho = (double *)dev_alloc(s, sizeof(double) * N);
    s->taps = dev_alloc(s, s->esz * (kMaxTaps + 1));
    if (!s->err || !s->dbuf || !s->rho || !s->taps || !s->jbox) {
      dev_free_all(s);
      delete s;
      return fail(RELPIC_ENOMEM, "create: allocation failed");
    }
    hipError_t e = hipSuccess;
    for (int k = 0; k < 10 && e == hipSuccess; ++k)
      if (s->F[k]) e = hipMemsetAsync(s->F[k], 0, s->esz * N, s->st);
    for (int d = 0; d < 3 && e == hipSuccess; ++d) e = hipMemsetAsync(s->Bx[d], 0, s->esz * N, s->st);
    for (int d = 0; d < 3 && e == hipSuccess; ++d)
      if (s->Ex[d]) e = hipMemsetAsync(s->Ex[d], 0, s->esz * N, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->err, 0, 64, s->st);
    if (e == hipSuccess) {
      launch_reset_box(s->jbox, s->st);
      launch_reset_box(s->jbox + 1, s->st);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      std::vector<unsigned char> host(s->esz * taps.size());
      for (size_t i = 0; i < taps.size(); ++i) {
        if (prec == RELPIC_FP32) {
          float v = (float)taps[i];
          std::memcpy(&host[i * 4], &v, 4);
        } else {
          std::memcpy(&host[i * 8], &taps[i], 8);
        }
      }
      e = hipMemcpyAsync(s->taps, host.data(), host.size(), hipMemcpyHostToDevice, s->st);
      if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) {
      dev_free_all(s);
      delete s;
      return fail(RELPIC_EDEVICE, std::string("create: ") + hipGetErrorString(e));
    }
    *out = s;
    return RELPIC_OK;
  });
}

relpic_status relpic_destroy(relpic_sim *sim) {
  return guarded("destroy", [&]() -> relpic_status {
    if (!sim) return RELPIC_OK;
    (void)hipStreamSynchronize(sim->st);
    for (hipEvent_t e : sim->ev_pool) (void)hipEventDestroy(e);
    dev_free_all(sim);
    delete sim;
    return RELPIC_OK;
  });
}

relpic_status relpic_add_species(relpic_sim *s, double q_over_m, double Q, int64_t capacity, int *species_id) {
  return guarded("add_species", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    // at most 2^32 bytes per particle array (the push addresses them with
    // 32-bit offsets)
    if (!std::isfinite(q_over_m) || !std::isfinite(Q) || capacity < 0 || capacity > (1LL << 32) / (int64_t)s->esz)
      return fail(RELPIC_EINVAL, "add_species: bad q/m, charge or capacity");
    Species sp;
    sp.qm = q_over_m;
    sp.Q = Q;
    sp.cap = capacity;
    const size_t cap = (size_t)std::max<int64_t>(capacity, 1);
    sp.cell = (int *)dev_alloc(s, sizeof(int) * cap);
    sp.cell2 = (int *)dev_alloc(s, sizeof(int) * cap);
    sp.id = (int *)dev_alloc(s, sizeof(int) * cap);
    sp.id2 = (int *)dev_alloc(s, sizeof(int) * cap);
    sp.keys = (unsigned *)dev_alloc(s, sizeof(unsigned) * cap);
    sp.keys2 = (unsigned *)dev_alloc(s, sizeof(unsigned) * cap);
    sp.idx = (unsigned *)dev_alloc(s, sizeof(unsigned) * cap);
    sp.idx2 = (unsigned *)dev_alloc(s, sizeof(unsigned) * cap);
    bool ok = sp.cell && sp.cell2 && sp.id && sp.id2 && sp.keys && sp.keys2 && sp.idx && sp.idx2;
    for (int d = 0; d < 3 && ok; ++d) {
      sp.o[d] = (d < s->ndim) ? dev_alloc(s, s->esz * cap) : nullptr;
      sp.o2[d] = (d < s->ndim) ? dev_alloc(s, s->esz * cap) : nullptr;
      sp.u[d] = dev_alloc(s, s->esz * cap);
      sp.u2[d] = dev_alloc(s, s->esz * cap);
      ok = (d >= s->ndim || (sp.o[d] && sp.o2[d])) && sp.u[d] && sp.u2[d];
    }
    if (!ok) return fail(RELPIC_ENOMEM, "add_species: allocation failed");
    s->sp.push_back(sp);
    if (species_id) *species_id = (int)s->sp.size() - 1;
    return RELPIC_OK;
  });
}

relpic_status relpic_load_particles(relpic_sim *s, int species, int64_t n, const int32_t *cell, const double *offset,
                                    const double *u) {
  return guarded("load_particles", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (species < 0 || species >= (int)s->sp.size()) return fail(RELPIC_EINVAL, "load: bad species");
    if (n < 0 || (n > 0 && (!cell || !offset || !u))) return fail(RELPIC_EINVAL, "load: bad arrays");
    Species &sp = s->sp[species];
    if (sp.n + n > sp.cap) return fail(RELPIC_ERANGE, "load: capacity exceeded");
    if (n == 0) return RELPIC_OK;
    const Geo g = make_geo(s);
    const int nd = s->ndim;
    // validate everything before the first byte is copied: a rejected load leaves the species unchanged
    for (int64_t i = 0; i < n; ++i) {
      long long l1 = cell[i * nd + 0];
      if (g.window) {
        l1 -= s->ws;
        if (l1 < 2 || l1 > s->n[0] - 3) return fail(RELPIC_ERANGE, "load: particle outside the window interior");
      } else if (l1 < 0 || l1 >= s->n[0]) {
        return fail(RELPIC_ERANGE, "load: x1 cell outside the grid");
      }
      const int c2 = cell[i * nd + 1];
      const int c3 = nd == 3 ? cell[i * nd + 2] : 0;
      if (c2 < 0 || c2 >= s->n[1] || c3 < 0 || c3 >= s->n[2]) return fail(RELPIC_ERANGE, "load: cell outside the grid");
      for (int d = 0; d < nd; ++d) {
        const double o = offset[i * nd + d];
        if (!(o >= -0.5 && o < 0.5)) return fail(RELPIC_EINVAL, "load: offset outside [-1/2, 1/2)");
      }
      for (int d = 0; d < 3; ++d)
        if (!std::isfinite(u[i * 3 + d])) return fail(RELPIC_EINVAL, "load: non-finite momentum");
    }
    // staged through bounded host buffers (kStage particles at a time)
    const int64_t chunk = std::min<int64_t>(n, kStage);
    std::vector<int> packed(chunk), ids(chunk);
    std::vector<unsigned char> col((size_t)chunk * s->esz);
    auto put = [&](void *dst_base, int64_t first, int64_t m, const double *src, int stride, int k) -> relpic_status {
      for (int64_t i = 0; i < m; ++i) {
        const double v = src[(first + i) * stride + k];
        if (s->prec == RELPIC_FP32) {
          const float x = (float)v;
          std::memcpy(&col[i * 4], &x, 4);
        } else {
          std::memcpy(&col[i * 8], &v, 8);
        }
      }
      HIP_OK(hipMemcpyAsync((char *)dst_base + s->esz * (sp.n + first), col.data(), s->esz * m, hipMemcpyHostToDevice,
                            s->st));
      HIP_OK(hipStreamSynchronize(s->st));
      return RELPIC_OK;
    };
    for (int64_t first = 0; first < n; first += chunk) {
      const int64_t m = std::min<int64_t>(chunk, n - first);
      for (int64_t i = 0; i < m; ++i) {
        const int64_t q = first + i;
        long long l1 = cell[q * nd + 0];
        if (g.window) l1 -= s->ws;
        const int c2 = cell[q * nd + 1];
        const int c3 = nd == 3 ? cell[q * nd + 2] : 0;
        const int cc = (int)((l1 + g.ws_mod) % s->n[0]);
        packed[i] = cc + s->n[0] * (c2 + s->n[1] * c3);
        ids[i] = (int)(sp.next_id + q);
      }
      HIP_OK(hipMemcpyAsync(sp.cell + sp.n + first, packed.data(), sizeof(int) * m, hipMemcpyHostToDevice, s->st));
      HIP_OK(hipMemcpyAsync(sp.id + sp.n + first, ids.data(), sizeof(int) * m, hipMemcpyHostToDevice, s->st));
      HIP_OK(hipStreamSynchronize(s->st));
      for (int d = 0; d < nd; ++d)
        if (relpic_status r = put(sp.o[d], first, m, offset, nd, d)) return r;
      for (int d = 0; d < 3; ++d)
        if (relpic_status r = put(sp.u[d], first, m, u, 3, d)) return r;
    }
    sp.n += n;
    sp.next_id += n;
    sp.dirty = true;
    return RELPIC_OK;
  });
}

relpic_status relpic_set_injection(relpic_sim *s, int species, const int *ppc, double uth, uint64_t seed) {
  return guarded("set_injection", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (species < 0 || species >= (int)s->sp.size() || !ppc) return fail(RELPIC_EINVAL, "injection: bad species");
    if (s->grid.bc1 != RELPIC_BC_WINDOW) return fail(RELPIC_ESTATE, "injection needs the moving window");
    Species &sp = s->sp[species];
    for (int d = 0; d < 3; ++d) {
      sp.ppc[d] = d < s->ndim ? ppc[d] : 1;
      if (sp.ppc[d] < 1 || sp.ppc[d] > 16) return fail(RELPIC_EINVAL, "injection: ppc must be in 1..16");
    }
    sp.inject = true;
    sp.uth = uth;
    sp.seed = seed;
    sp.inj_count = 0;
    return RELPIC_OK;
  });
}

relpic_status relpic_set_background_rho(relpic_sim *s, const double *rho, int64_t count) {
  return guarded("set_background_rho", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (!rho || count != s->N) return fail(RELPIC_EINVAL, "background: count must equal the number of cells");
    if (!s->rho_bg) {
      s->rho_bg = (double *)dev_alloc(s, sizeof(double) * s->N);
      if (!s->rho_bg) return fail(RELPIC_ENOMEM, "background: allocation failed");
    }
    // window-relative -> storage layout
    std::vector<double> st((size_t)s->N);
    const int n1 = s->n[0];
    const int wsm = make_geo(s).ws_mod;
    for (long long r = 0; r < s->N / n1; ++r)
      for (int l = 0; l < n1; ++l) st[r * n1 + (l + wsm) % n1] = rho[r * n1 + l];
    HIP_OK(hipMemcpyAsync(s->rho_bg, st.data(), sizeof(double) * s->N, hipMemcpyHostToDevice, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    return RELPIC_OK;
  });
}

relpic_status relpic_step(relpic_sim *s, int64_t nsteps) {
  return guarded("step", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (nsteps < 0) return fail(RELPIC_EINVAL, "step: negative count");
    if (s->prec == RELPIC_FP32) return do_steps<float>(s, nsteps);
    return do_steps<double>(s, nsteps);
  });
}

relpic_status relpic_sync(relpic_sim *s) {
  return guarded("sync", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    int err = 0;
    HIP_OK(hipMemcpyAsync(&err, s->err, sizeof(int), hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    if (err) {
      char buf[96];
      std::snprintf(buf, sizeof buf, "kernel error word 0x%x (1: moved > 1 cell, 2: NaN momentum)", err);
      return fail(RELPIC_EDEVICE, buf);
    }
    return RELPIC_OK;
  });
}

relpic_status relpic_read_field(relpic_sim *s, relpic_field f, double *host, int64_t count) {
  return guarded("read_field", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if ((int)f < 0 || (int)f > 8 || !host || count != s->N) return fail(RELPIC_EINVAL, "read_field: bad field or count");
    return copy_rows(s, (int)f, host, true);
  });
}

relpic_status relpic_write_field(relpic_sim *s, relpic_field f, const double *host, int64_t count) {
  return guarded("write_field", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if ((int)f < 0 || (int)f > 8 || !host || count != s->N) return fail(RELPIC_EINVAL, "write_field: bad field or count");
    return copy_rows(s, (int)f, const_cast<double *>(host), false);
  });
}

relpic_status relpic_field_device_ptr(relpic_sim *s, relpic_field f, void **ptr, int *elem_bytes) {
  return guarded("field_device_ptr", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if ((int)f < 0 || (int)f > 8 || !ptr) return fail(RELPIC_EINVAL, "field_device_ptr: bad field");
    *ptr = s->F[(int)f];
    if (elem_bytes) *elem_bytes = (int)s->esz;
    return RELPIC_OK;
  });
}

relpic_status relpic_read_particles(relpic_sim *s, int species, int64_t cap, int32_t *cell, double *offset, double *u,
                                    uint8_t *alive, int64_t *id, int64_t *n_out) {
  return guarded("read_particles", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (species < 0 || species >= (int)s->sp.size()) return fail(RELPIC_EINVAL, "read_particles: bad species");
    Species &sp = s->sp[species];
    if (n_out) *n_out = sp.n;
    if (cap < sp.n || !cell || !offset || !u || !alive) return fail(RELPIC_ERANGE, "read_particles: buffers too small");
    const long long n = sp.n;
    const int nd = s->ndim;
    const int n1 = s->n[0];
    const int wsm = make_geo(s).ws_mod;
    // staged through bounded host buffers (kStage particles at a time)
    const long long chunk = std::max<long long>(1, std::min<long long>(n, kStage));
    std::vector<int> packed(chunk), ids(chunk);
    std::vector<unsigned char> raw(s->esz * chunk);
    for (long long first = 0; first < n; first += chunk) {
      const long long m = std::min(chunk, n - first);
      auto get = [&](const void *src, int stride_idx, int stride, double *dst) -> relpic_status {
        HIP_OK(hipMemcpyAsync(raw.data(), (const char *)src + s->esz * first, s->esz * m, hipMemcpyDeviceToHost, s->st));
        HIP_OK(hipStreamSynchronize(s->st));
        for (long long i = 0; i < m; ++i) {
          double v;
          if (s->esz == 4) {
            float x;
            std::memcpy(&x, &raw[i * 4], 4);
            v = x;
          } else {
            std::memcpy(&v, &raw[i * 8], 8);
          }
          dst[(first + i) * stride + stride_idx] = v;
        }
        return RELPIC_OK;
      };
      HIP_OK(hipMemcpyAsync(packed.data(), sp.cell + first, sizeof(int) * m, hipMemcpyDeviceToHost, s->st));
      HIP_OK(hipMemcpyAsync(ids.data(), sp.id + first, sizeof(int) * m, hipMemcpyDeviceToHost, s->st));
      for (int d = 0; d < nd; ++d)
        if (relpic_status r = get(sp.o[d], d, nd, offset)) return r;
      for (int d = 0; d < 3; ++d)
        if (relpic_status r = get(sp.u[d], d, 3, u)) return r;
      for (long long i = 0; i < m; ++i) {
        const long long q = first + i;
        const int pk = packed[i];
        alive[q] = pk >= 0 ? 1 : 0;
        if (id) id[q] = ids[i];
        if (pk < 0) {
          for (int d = 0; d < nd; ++d) cell[q * nd + d] = 0;
          continue;
        }
        const int s1 = pk % n1;
        const int rest = pk / n1;
        const int l1 = ((s1 - wsm) % n1 + n1) % n1;
        cell[q * nd + 0] = (int32_t)(l1 + (s->grid.bc1 == RELPIC_BC_WINDOW ? s->ws : 0));
        cell[q * nd + 1] = rest % s->n[1];
        if (nd == 3) cell[q * nd + 2] = rest / s->n[1];
      }
    }
    return RELPIC_OK;
  });
}

relpic_status relpic_gather_particles(relpic_sim *s, int species, int64_t first, int64_t count, double *EB) {
  return guarded("gather_particles", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (species < 0 || species >= (int)s->sp.size()) return fail(RELPIC_EINVAL, "gather_particles: bad species");
    Species &sp = s->sp[species];
    if (first < 0 || count < 0 || first + count > sp.n) return fail(RELPIC_ERANGE, "gather_particles: slots out of range");
    if (count > 0 && !EB) return fail(RELPIC_EINVAL, "gather_particles: null output");
    if (count == 0) return RELPIC_OK;
    const long long chunk = std::min<long long>(count, 1LL << 20);
    if (chunk > s->gather_cap) {
      s->gather_buf = (double *)dev_alloc(s, sizeof(double) * 6 * (size_t)chunk);
      if (!s->gather_buf) return fail(RELPIC_ENOMEM, "gather_particles: allocation failed");
      s->gather_cap = chunk;
    }
    const Geo g = make_geo(s);
    for (long long k0 = 0; k0 < count; k0 += chunk) {
      const long long m = std::min<long long>(chunk, count - k0);
      if (s->prec == RELPIC_FP32)
        launch_gather_at_particles<float>(s->ndim, g, fields<float>(s), parts<float>(sp), first + k0, m, s->gather_buf,
                                          s->st);
      else
        launch_gather_at_particles<double>(s->ndim, g, fields<double>(s), parts<double>(sp), first + k0, m,
                                           s->gather_buf, s->st);
      HIP_OK(hipGetLastError());
      HIP_OK(hipMemcpyAsync(EB + 6 * k0, s->gather_buf, sizeof(double) * 6 * m, hipMemcpyDeviceToHost, s->st));
      HIP_OK(hipStreamSynchronize(s->st));
    }
    return RELPIC_OK;
  });
}

relpic_status relpic_e1_residual(relpic_sim *s, int species, int64_t slot, const relpic_kspace *q, int64_t npts,
                                 const int32_t *i1_rel, double *sim_out, double *theory_out) {
  return guarded("e1_residual", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (species < 0 || species >= (int)s->sp.size()) return fail(RELPIC_EINVAL, "e1_residual: bad species");
    Species &sp = s->sp[species];
    if (slot < 0 || slot >= sp.n) return fail(RELPIC_ERANGE, "e1_residual: particle slot out of range");
    if (!q || npts < 1 || npts > 4096 || !i1_rel || !sim_out || !theory_out)
      return fail(RELPIC_EINVAL, "e1_residual: bad arguments");
    // the theory must describe this run: its axial operator, kappa = dx1/dt and r = dx2/dx1
    const double kappa = s->dx[0] / s->grid.dt, r = s->dx[1] / s->dx[0];
    if (std::fabs(q->kappa - kappa) > 1e-9 * kappa || std::fabs(q->r - r) > 1e-9 * r)
      return fail(RELPIC_EINVAL, "e1_residual: kappa or r differ from the simulation's");
    // operators of q, zero-padded like the simulation's, must equal them
    auto coef = [](int Mq, const double *Cq, int l) { return l < Mq ? ((Mq == 1 && !Cq) ? 1.0 : Cq[l]) : 0.0; };
    if (q->M > s->M || q->MB > s->M || q->MB < 0)
      return fail(RELPIC_EINVAL, "e1_residual: axial operator differs from the simulation's");
    for (int l = 0; l < s->M; ++l) {
      const double ce = coef(q->M, q->C, l);
      const double cb = q->MB > 0 ? coef(q->MB, q->CB, l) : ce;
      if (ce != s->C[l] || cb != s->CB[l])
        return fail(RELPIC_EINVAL, "e1_residual: axial coefficients differ from the simulation's");
    }
    // the particle: on a node along x1 (the k-space field is for a charge on a node)
    int packed = -1;
    unsigned char o1raw[8] = {};
    HIP_OK(hipMemcpyAsync(&packed, sp.cell + slot, sizeof(int), hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipMemcpyAsync(o1raw, (const char *)sp.o[0] + s->esz * slot, s->esz, hipMemcpyDeviceToHost, s->st));
    HIP_OK(hipStreamSynchronize(s->st));
    if (packed < 0) return fail(RELPIC_ESTATE, "e1_residual: the particle has been dropped");
    double o1;
    if (s->esz == 4) {
      float x;
      std::memcpy(&x, o1raw, 4);
      o1 = x;
    } else {
      std::memcpy(&o1, o1raw, 8);
    }
    if (std::fabs(o1) > 1e-6) return fail(RELPIC_ERANGE, "e1_residual: the particle is not on an x1 node");
    const int n1 = s->n[0];
    const Geo g = make_geo(s);
    const int s1 = packed % n1, row = packed / n1;
    const int c1 = ((s1 - g.ws_mod) % n1 + n1) % n1;  // window cell
    std::vector<double> line((size_t)n1);
    {
      std::vector<unsigned char> raw((size_t)n1 * s->esz);
      HIP_OK(hipMemcpyAsync(raw.data(), (const char *)s->F[0] + (size_t)row * n1 * s->esz, raw.size(),
                            hipMemcpyDeviceToHost, s->st));
      HIP_OK(hipStreamSynchronize(s->st));
      for (int l = 0; l < n1; ++l) {
        const int sc = (l + g.ws_mod) % n1;
        if (s->esz == 4) {
          float x;
          std::memcpy(&x, &raw[(size_t)sc * 4], 4);
          line[l] = x;
        } else {
          std::memcpy(&line[l], &raw[(size_t)sc * 8], 8);
        }
      }
    }
    std::vector<double> rel((size_t)npts);
    // E1 dx1 / Q in 2D, E1 dx1^2 / Q in 3D (the k-space field's normalization)
    const double scale = (s->ndim == 3 ? s->dx[0] * s->dx[0] : s->dx[0]) / sp.Q;
    for (int64_t k = 0; k < npts; ++k) {
      long long l = (long long)c1 + i1_rel[k];
      if (s->grid.bc1 == RELPIC_BC_WINDOW) {
        if (l < 0 || l >= n1) return fail(RELPIC_ERANGE, "e1_residual: point outside the window");
      } else {
        l = ((l % n1) + n1) % n1;
      }
      sim_out[k] = line[(size_t)l] * scale;
      rel[(size_t)k] = (double)i1_rel[k];
    }
    relpic_kspace qq = *q;
    relpic_device dv = s->dev;
    if (s->ndim == 2) return relpic_kspace_e1(&qq, &dv, npts, rel.data(), theory_out);
    // 3D: the particle's own (x2, x3) row of the 3D field (Eq. 9 with both transverse integrals)
    const std::vector<int32_t> zero((size_t)npts, 0);
    return relpic_kspace_field(&qq, &dv, 3, s->dx[2] / s->dx[0], npts, rel.data(), zero.data(), zero.data(),
                               theory_out);
  });
}

relpic_status relpic_diagnostics(relpic_sim *s, relpic_diag *out) {
  return guarded("diagnostics", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (!out) return fail(RELPIC_EINVAL, "diagnostics: null output");
    if (s->prec == RELPIC_FP32) return do_diag<float>(s, out);
    return do_diag<double>(s, out);
  });
}

relpic_status relpic_get_step(relpic_sim *s, int64_t *step, int64_t *window_start) {
  return guarded("get_step", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (step) *step = s->step;
    if (window_start) *window_start = s->ws;
    return RELPIC_OK;
  });
}

relpic_status relpic_sort_particles(relpic_sim *s) {
  return guarded("sort_particles", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    for (auto &sp : s->sp) {
      relpic_status r = s->prec == RELPIC_FP32 ? do_sort<float>(s, sp) : do_sort<double>(s, sp);
      if (r) return r;
    }
    return RELPIC_OK;
  });
}

relpic_status relpic_set_sort_interval(relpic_sim *s, int64_t interval) {
  return guarded("set_sort_interval", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (interval < 0) return fail(RELPIC_EINVAL, "sort interval must be >= 0");
    s->sort_interval = interval;
    return RELPIC_OK;
  });
}

relpic_status relpic_set_current_filter(relpic_sim *s, int npass, double comp) {
  return guarded("set_current_filter", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (npass < 0 || npass > 16) return fail(RELPIC_EINVAL, "current filter: npass must be in 0..16");
    if (npass > 0 && !std::isfinite(comp)) return fail(RELPIC_EINVAL, "current filter: compensator must be finite");
    if (npass > 0 && s->n[0] > kFilterMaxLine)
      return fail(RELPIC_EINVAL, "current filter: n1 exceeds the longest line it stages (4096)");
    s->filt_npass = npass;
    s->filt_comp = npass > 0 ? comp : 0.0;
    return RELPIC_OK;
  });
}

relpic_status relpic_set_fused_fields(relpic_sim *s, int enable, int *active) {
  return guarded("set_fused_fields", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (enable && !s->Ex[0]) {
      if (active) *active = 0;
      return fail(RELPIC_EINVAL, "fused field update: not available on this grid (3D, n1 <= 512, n2 even, n1 at "
                                 "least twice the staged halo)");
    }
    s->fuse = enable != 0;
    if (active) *active = s->fuse ? 1 : 0;
    return RELPIC_OK;
  });
}

relpic_status relpic_profile_enable(relpic_sim *s, int on) {
  return guarded("profile_enable", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    HIP_OK(hipStreamSynchronize(s->st));
    s->prof = on != 0;
    s->ev_used = 0;
    s->ev_marks.clear();
    return RELPIC_OK;
  });
}

relpic_status relpic_profile_read(relpic_sim *s, relpic_profile *out) {
  return guarded("profile_read", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (!out) return fail(RELPIC_EINVAL, "profile_read: null output");
    HIP_OK(hipStreamSynchronize(s->st));
    for (int k = 0; k < RELPIC_NUM_KERNEL_CLASSES; ++k) {
      out->launches[k] = 0;
      out->total_ms[k] = 0.0;
    }
    for (auto &m : s->ev_marks) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, s->ev_pool[m.second], s->ev_pool[m.second + 1]));
      out->launches[m.first % 64] += 1;
      out->total_ms[m.first % 64] += ms;
    }
    return RELPIC_OK;
  });
}

relpic_status relpic_profile_read_species(relpic_sim *s, int species, int64_t *launches, double *total_ms) {
  return guarded("profile_read_species", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (species < 0 || species >= (int)s->sp.size() || !launches || !total_ms)
      return fail(RELPIC_EINVAL, "profile_read_species: bad species or output");
    HIP_OK(hipStreamSynchronize(s->st));
    *launches = 0;
    *total_ms = 0.0;
    for (auto &m : s->ev_marks) {
      if (m.first != 64 * (species + 1)) continue;
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, s->ev_pool[m.second], s->ev_pool[m.second + 1]));
      *launches += 1;
      *total_ms += ms;
    }
    return RELPIC_OK;
  });
}

relpic_status relpic_correction_halfwidth(relpic_sim *s, int *hw) {
  return guarded("correction_halfwidth", [&]() -> relpic_status {
    if (relpic_status r = check_sim(s)) return r;
    if (hw) *hw = s->ng;
    return RELPIC_OK;
  });
}

}  // extern "C"
