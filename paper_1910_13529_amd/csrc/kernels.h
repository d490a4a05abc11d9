// Launch entry points of the relpic HIP kernels (internal to the library).
#pragma once

#include "relpic_internal.h"

namespace relpic {

template <typename Real>
struct PushParams {
  Real half_qmdt;  // (q/m) dt / 2
  Real dtdx[3];    // dt / dx_d
  Real f1, f2, f3; // -Q dx_d / (dV dt): Esirkepov current factors
  Real fv;         // Q / dV: out-of-plane current factor (2D)
  int shift;       // 1 if the window advances after this step
};

// Bout = Bin - curl+ E with the time factor folded into ax, h2, h3
template <typename Real>
void launch_curl_e(int ndim, const Geo &g, const Fields<Real> &f, Real *const Bin[3], Real *const Bout[3],
                   const Axial<Real> &ax, Real h2, Real h3, hipStream_t st);
// E += curl- B (f.B*), time factor folded into ax, e2, e3
template <typename Real>
void launch_curl_b(int ndim, const Geo &g, const Fields<Real> &f, const Axial<Real> &ax, Real e2, Real e3,
                   hipStream_t st);
// E -= dt J inside the J box (x1 widened by pad), J cleared there, `next` box reset
template <typename Real>
void launch_add_j(const Geo &g, const Fields<Real> &f, const Real *J1src, Real dt, const JBox *box, int pad,
                  JBox *next, hipStream_t st);
template <typename Real>
void launch_jcorr(const Geo &g, const Real *J1, Real *J1c, const Real *taps, int ng, const JBox *box,
                  hipStream_t st);
// Current filter along x1, in place on each non-null array: npass passes of
// (1/4, 1/2, 1/4) and one of (ca, cb, ca), over the x1 lines of the box
// (box null: every line of the grid).  Input: the box's x1 range widened by
// in_pad, taken as zero outside it; output: that range widened by npass + 1.
constexpr int kFilterMaxLine = 4096;  // longest x1 line (n1) the filter stages in LDS
template <typename Real>
void launch_filter_rows(const Geo &g, Real *A0, Real *A1, Real *A2, const JBox *box, int in_pad, int npass, Real ca,
                        Real cb, hipStream_t st);
// new leading slab after a window shift: E = 0, B (f.B*, at n + 1/2) such
// that B^{n+1} = 0 there, other B buffer Bx cleared
template <typename Real>
void launch_new_slab(const Geo &g, const Fields<Real> &f, Real *const Bx[3], int col, const Axial<Real> &ax,
                     hipStream_t st);
void launch_reset_box(JBox *b, hipStream_t st);
// window shift after a fused step: E (E^{n+1}), X (B^{n+1/2}) and Y (the B
// the fused update produced with factor f) from the old window to the
// shifted one; ch: C_l (dt/2) / dx1, f2m1 = 2 f - 1
template <typename Real>
void launch_shift_fused(const Geo &g, Real *const E[3], Real *const X[3], Real *const Y[3], int col,
                        const Axial<Real> &ch, Real f2m1, hipStream_t st);
// J cleared inside the J box (x1 widened by pad), `next` box reset
template <typename Real>
void launch_clear_j(const Geo &g, const Fields<Real> &f, const JBox *box, int pad, JBox *next, hipStream_t st);

// Fused 3D update: Eout = Ein + dt curl- B - dt J (inside the box; J1s is J1
// or the corrected J1c), then Bout = B - curl+ Eout with the time factor
// folded into axB, h2, h3; axE, e2c, e3c carry dt.  Ein, Eout, B, Bout
// distinct.  Only for grids where leap_supported holds.
template <typename Real>
bool leap_supported(const Geo &g, int M);
template <typename Real>
void launch_leap(const Geo &g, Real *const Ein[3], Real *const Eout[3], Real *const B[3], Real *const Bout[3],
                 const Real *J1s, const Real *J2, const Real *J3, const JBox *box, int pad, Real dt,
                 const Axial<Real> &axE, Real e2c, Real e3c, const Axial<Real> &axB, Real h2, Real h3,
                 hipStream_t st);

// K particles per thread; each workgroup handles a contiguous chunk of
// 256 * K particles (sorted by cell for the LDS-tiled deposit to pay off);
// Push chunks: one per sort tile of the last tile sort ([first[t], end[t])
// of the array, ntiles of them, covering the first nsorted particles), then
// runs of 256 K particles over the rest (appended since); ntiles = nsorted =
// 0: runs of 256 K over the whole array.
struct PushChunks {
  const int *first = nullptr, *end = nullptr;
  long long ntiles = 0, nsorted = 0;
  int K = 1;
};
// workgroups (and scratch boxes) of a push over n particles
long long push_grid(const PushChunks &pc, long long n);
// wide (3D, FP32): deposit rounds over boxes four x1 cells wide instead of
// two, and cell groups, for species spread over the grid at a few particles
// per cell; long_runs (with wide): the cells hold runs of several particles,
// so lanes outside the cell groups deposit directly instead of in rounds;
// blockbox: push_grid(pc, n) scratch boxes, merged into *jbox after the
// launch
template <typename Real>
void launch_push_deposit(int ndim, const Geo &g, const Fields<Real> &f, const HalfB<Real> &Bh,
                         const Particles<Real> &p, const PushParams<Real> &q, const PushChunks &pc, bool wide,
                         bool long_runs, JBox *blockbox, int *err, hipStream_t st);
// *jbox = union of the nbox per-workgroup boxes (atomic min/max into *jbox)
void launch_merge_boxes(const JBox *blockbox, long long nbox, JBox *jbox, hipStream_t st);
long long push_blocks(long long n, int K);

// ---- particle sort by cell ------------------------------------------------------
// keys[i] = sort key of particle i's cell (dropped particles: 0xFFFFFFFF),
// idx[i] = i; tiles = 0: the packed cell index, t > 0: 2^t x 4 x 4 tiles of
// cells (2D: 2^t x 4), x1 fastest inside a tile
template <typename Real>
void launch_sort_keys(const Geo &g, const Particles<Real> &p, int tiles, unsigned *keys, unsigned *idx,
                      hipStream_t st);
// whether the tiled sort keys (any t <= 3) fit in 32 bits on this grid
bool sort_tiles_fit(const Geo &g);
// dst[j] = src[perm[j]] for j below src.n and, when count is given, below
// *count (device word)
template <typename Real>
void launch_permute(const Particles<Real> &src, const Particles<Real> &dst, const int *id_src, int *id_dst,
                    const unsigned *perm, int ndim, hipStream_t st, const unsigned long long *count = nullptr);
// index range of each sort tile (key >> shift) among the n alive particles
// of a tile-sorted key array; first, end: ntiles ints each, cleared by the
// caller
void launch_tile_ranges(const unsigned *keys, long long n, int shift, long long ntiles, int *first, int *end,
                        hipStream_t st);
// Counting sort of (key, index) pairs with keys below nkeys (others, the
// dropped particles, left out): keys_out / idx_out receive the totals[0]
// alive pairs in key order (unordered inside a key), totals[1] = distinct
// keys.  count: nkeys words cleared by the caller (left holding the bucket
// ends); bsum, bocc: key_scan_blocks(nkeys) entries of scratch.
long long key_scan_blocks(unsigned nkeys);
void launch_key_sort(const unsigned *keys, long long n, unsigned nkeys, unsigned *count, unsigned long long *bsum,
                     unsigned *bocc, unsigned long long *totals, unsigned *keys_out, unsigned *idx_out,
                     hipStream_t st);
// sorted keys: distinct alive cells added to *runs, alive count written to *alive
void launch_count_runs(const unsigned *keys, long long n, unsigned long long *runs, unsigned long long *alive,
                       hipStream_t st);
// radix sort of (key, index) pairs; temp/temp_bytes from a first call with temp = null
hipError_t sort_pairs(void *temp, size_t &temp_bytes, const unsigned *keys_in, unsigned *keys_out,
                      const unsigned *idx_in, unsigned *idx_out, long long n, hipStream_t st);

// ---- FP64 diagnostics ----------------------------------------------------------
// acc[0] += 1/2 sum (E^2 + B^2)
template <typename Real>
void launch_diag_field_energy(const Geo &g, const Fields<Real> &f, double *acc, hipStream_t st);
// acc[0] += sum Q/(q/m) (gamma - 1); cnt[0] += alive particles
template <typename Real>
void launch_diag_kinetic(const Particles<Real> &p, double mass, double *acc, unsigned long long *cnt,
                         hipStream_t st);
// rho (FP64, storage layout) += Q S(x_p)/dV for every alive particle
template <typename Real>
void launch_diag_rho(int ndim, const Geo &g, const Particles<Real> &p, double qdv, double *rho, hipStream_t st);
// max |d- . E - rho - rho_bg| over interior nodes, max |rho| of the particles, sum rho
// (rho_bg window-relative, may be null); out[0..2] hold the FP64 results
template <typename Real>
void launch_diag_gauss(int ndim, const Geo &g, const Fields<Real> &f, const Axial<double> &c1dx, double idx2,
                       double idx3, const double *rho, const double *rho_bg, int margin1, double *out,
                       hipStream_t st);

// E^n, B^n (f.B* = canonical B^n) at particles first .. first + count - 1,
// quadratic spline per staggered component, FP64 out[6 k + c] (dropped: 0)
template <typename Real>
void launch_gather_at_particles(int ndim, const Geo &g, const Fields<Real> &f, const Particles<Real> &p,
                                long long first, long long count, double *out, hipStream_t st);

// ---- plasma injection ------------------------------------------------------------
// 3D stores the slab's cells in kInjBlock x kInjBlock transverse blocks, 2D
// in row order; ids and momenta follow the row order either way
constexpr int kInjBlock = 8;
template <typename Real>
void launch_inject_slab(int ndim, const Geo &g, Particles<Real> p, int *id, long long first, int win_cell, int ppc1,
                        int ppc2, int ppc3, double uth, unsigned long long seed, unsigned long long counter0,
                        long long id0, hipStream_t st);

}  // namespace relpic
