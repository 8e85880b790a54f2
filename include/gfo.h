/*
 * gfo.h - C ABI of libgfo, the MI355X (gfx950) Green's-function pixel-by-pixel
 * greedy optimiser.
 *
 * Problem (paper Sec. II, eq. form1): N design pixels of area h^2 on an
 * ny x nx grid, a table of permittivities, n_mon monitor points, and a figure
 * of merit FOM = |E(r_m0)|^2 at one monitor.  2-D TM (scalar E_z) reduction of
 * the paper's 3-D dyadic formalism; background vacuum.
 *
 * Stored state of the current structure (all in caller-owned DEVICE memory):
 *   G      R x N complex matrix, R = N + n_mon, row-major with leading
 *          dimension ldG (elements).  Rows: design pixels p = iy*nx + ix, then
 *          monitors.  Columns: design pixels.  G is "area included": entry
 *          (r, q) is h^2 times the two-point Green's function (diagonal: its
 *          integral over the pixel), so a contrast alpha = k0^2 (eps' - eps)
 *          plays the role of the paper's b = k0^2 d_eps dV (eq. form4).
 *   E      R complex field values, same element type as G.
 *   diag64 N complex128 values: FP64 copy of diag(G) used for every
 *          denominator 1 - alpha G_pp (the only FP64 state besides refresh).
 *   eps_idx N uint8: material index of each pixel into the permittivity table.
 *   flips  (pixel, eps_idx) history of accepted moves, 2*flip_cap int32.
 * Complex numbers are interleaved {re, im}: float2 for GFO_C64, double2 for
 * GFO_C128.
 *
 * Conventions common to every entry point:
 *   - Pointers are device pointers unless their name starts with h_ (host).
 *   - The library never allocates or frees caller memory and keeps no pointer
 *     after a call returns.  Scratch lives in the caller's workspace
 *     (gfo_workspace_size).
 *   - Calls only enqueue work on `stream` and return; results are visible
 *     after the stream is synchronised.  Exceptions are stated per function.
 *   - Return value: GFO_OK (0) or a negative error detected on the host:
 *     GFO_EINVAL (bad sizes or null pointers), GFO_EHIP (a HIP call failed),
 *     GFO_ENOSPC (workspace too small), GFO_ERANGE (refresh_G: more flipped
 *     pixels than kmax), GFO_ESCRATCH (score_candidates_static: problem
 *     larger than the static scratch).  Conditions met on the device are OR-ed
 *     into *state->status (GFO_STATUS_*), to be read by the caller when it
 *     synchronises.  The library never aborts the process.
 *   - GFO_EHIP names a failure of the call's own HIP calls or launches
 *     (gfo_last_hip_error gives the HIP code).  An entry point that launches
 *     kernels first reads and drops the thread's pending HIP error, one left
 *     by an earlier failed call of the caller or of another library.
 */
#ifndef GFO_H
#define GFO_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GFO_C64 = 0, GFO_C128 = 1 };            /* storage type of G and E */
enum { GFO_FP32 = 0, GFO_BF16 = 1 };           /* MFMA input type of the rank-k update */
enum { GFO_OK = 0, GFO_EINVAL = -1, GFO_EHIP = -2, GFO_ENOSPC = -3, GFO_ERANGE = -4,
       GFO_ESCRATCH = -5 };
enum {                                         /* bits of the device status word */
  GFO_STATUS_SINGULAR = 1,      /* |1 - alpha G_jj| < 1e-12: move refused */
  GFO_STATUS_NONFINITE = 2,     /* a candidate score was NaN or infinite */
  GFO_STATUS_HISTORY_FULL = 4,  /* flip history at capacity: later moves not recorded */
  GFO_STATUS_REFRESH_OVERFLOW = 8 /* more flipped pixels than the refresh workspace holds */
};
#define GFO_MAX_EPS 8                          /* permittivity table entries */
#define GFO_MAX_RANK_K 32                      /* largest k of apply_flips_rank_k */
#define GFO_MAX_DELAY 128                      /* largest number of deferred rank-1 moves */
#define GFO_STATIC_SCRATCH_BYTES (8u << 20)    /* device scratch of score_candidates_static */

/* Problem description, read during a call, not retained. */
typedef struct {
  int32_t ny, nx, n_mon;        /* design rows (along y, the propagation axis), columns, monitors */
  int32_t dtype;                /* GFO_C64 or GFO_C128 */
  double wavelength, pitch;     /* lambda and pixel side h (same length unit) */
  double eps_bg;                /* background permittivity; must appear in the table */
  const double* h_mon_xy;       /* 2*n_mon monitor coordinates {x, y} (host) */
  int32_t fom_monitor;          /* index m0 of the FOM monitor */
  int32_t n_eps;                /* entries of the permittivity table, 2..GFO_MAX_EPS */
  const double* h_eps_table;    /* permittivity table (host) */
} gfo_problem;

/* Caller-owned device buffers of one optimisation job. */
typedef struct {
  void* G; int64_t ldG;         /* R x N, ldG >= N and a multiple of 64 (row stride; with
                                   packed, see below), gfo_g_elems() entries */
  void* E;                      /* R */
  double* diag64;               /* 2*N doubles */
  uint8_t* eps_idx;             /* N */
  int32_t* flips;               /* 2*flip_cap int32: (pixel, eps_idx) per accepted move */
  int32_t flip_cap;
  int32_t* n_flips;             /* 1 int32: moves accepted so far */
  int32_t kmax;                 /* largest flipped set refresh_G supports */
  void* work; size_t work_bytes;/* scratch, at least gfo_workspace_size() bytes, 256-B aligned */
  int32_t* status;              /* 1 int32 device status word (GFO_STATUS_* bits) */
  int32_t delay;                /* 0: eager rank-1 updates; 1..GFO_MAX_DELAY: deferred (see apply_flip) */
  int32_t pending_calls;        /* host counter kept by the library; set 0 before init_G0 */
  int32_t lower_stale;          /* host flag kept by the library: 1 while the strict lower
                                   triangle of the design block is out of date (see
                                   gfo_sync_lower); 0 or 1.  Before init_G0 (and refresh_G)
                                   set 0, or 1 to keep the upper triangle alone in eager
                                   mode too: the rank-1 update then skips the tiles below
                                   the diagonal, about half its HBM traffic */
  int32_t packed;               /* 0: dense R x ldG rows.  1: band-packed upper triangle of the
                                   design block (it is symmetric: Sec. II, reciprocity), about
                                   half the entries: design rows in bands of 64, the rows of
                                   band b holding columns [64 b, ldG) only and ldG - 64 b
                                   entries apart, band b starting at entry
                                   64 (b ldG - 32 b (b - 1)); then the N_m monitor rows, ldG
                                   apart.  Needs deferred updates (delay >= 1; else every call
                                   returns GFO_EINVAL); apply_flips_rank_k and gfo_sync_lower
                                   refuse it (GFO_EINVAL).  Set before init_G0, kept after */
} gfo_state;

/* One selected move.  pixel = -1 is the sentinel "no move improves the FOM". */
typedef struct {
  int32_t pixel, eps_idx;       /* flipped pixel and its new material index */
  double fom_new;               /* predicted FOM after the move */
  double dfom;                  /* fom_new minus the FOM before the move */
} gfo_pick;

/* Library version string. */
const char* gfo_version(void);

/* Human-readable text of a return code. */
const char* gfo_strerror(int code);

/* The HIP result behind the calling thread's most recent GFO_EHIP: the code of
 * the last HIP runtime call or kernel launch of the library that failed on
 * this thread (0 = none since the previous query), and its name in *h_name
 * (a static string; h_name may be NULL).  Clears the record.  Host only. */
int32_t gfo_last_hip_error(const char** h_name);

/* Bytes of workspace that a job of this problem needs with leading dimension
 * ldG (0: gfo_min_ld; else at least that and a multiple of 64) when refresh_G
 * must support up to kmax flipped pixels (kmax = 0: no refresh).  Host only. */
int gfo_workspace_size(const gfo_problem* prob, int64_t ldG, int32_t kmax, size_t* h_bytes);

/* Smallest valid leading dimension of G for this problem (N rounded up to 64). */
int64_t gfo_min_ld(const gfo_problem* prob);

/* Entries of G (of the problem's storage type) that a state with leading
 * dimension ldG (0: gfo_min_ld) needs: R x ldG dense (packed = 0), or the
 * band-packed design triangle and the monitor rows (packed = 1, see
 * gfo_state.packed).  Host only; GFO_EINVAL on a bad ldG or packed value. */
int gfo_g_elems(const gfo_problem* prob, int64_t ldG, int32_t packed, int64_t* h_elems);

/* Byte offset, inside the workspace, of the FP64 score array that
 * score_candidates fills: N x n_eps values in (pixel, eps_idx) row-major
 * order, -inf where (pixel, eps_idx) is not a candidate (and, after a call
 * with topk > 1, where the spacing rule excluded it).  Host only; for
 * inspection and tests. */
int gfo_scores_offset(const gfo_problem* prob, int64_t ldG, int32_t kmax, size_t* h_offset);

/* init_G0 - Green's matrix and field of the vacuum reference structure
 * (paper Sec. II: an analytic G0 is the starting point; Sec. IV starts from
 * vacuum).  Writes
 *   G[p, q] = h^2 (i/4) H0^(1)(k0 |r_p - r_q|)  (p != q; p a pixel or monitor)
 *   G[q, q] = (i pi a / (2 k0)) H1^(1)(k0 a) - 1/k0^2,  a = h / sqrt(pi)
 * (the kernel integrated over the equal-area disk), E = exp(i k0 y),
 * diag64 = diag(G) in FP64, eps_idx = index of eps_bg, n_flips = 0,
 * status = 0, and the FP64 offset table in the workspace that refresh_G
 * reuses.  Pixel centres: x = (ix - (nx-1)/2) h, y = (iy - (ny-1)/2) h.
 * All Hankel values are evaluated in FP64 and rounded once to the storage
 * type.  In deferred mode (state.delay > 0) the design block is written on
 * and above its diagonal only and state.lower_stale is set (gfo_sync_lower
 * completes it); otherwise the whole matrix is written and the flag cleared.
 * Exception to asynchrony: copies h_mon_xy to the workspace and synchronises
 * `stream` before returning, so the caller's host array need not outlive the
 * call. */
int init_G0(const gfo_problem* prob, gfo_state* st, hipStream_t stream);

/* score_candidates - score every candidate move and select (paper Sec. II A:
 * eqs. form4-form9 with a one-pixel region, evaluated at the monitor as in
 * eq. para1; selection as in Sec. IV/V: largest FOM increase, stop when none).
 * For every pixel p and every table entry e with bit e set in cand_mask and
 * e != eps_idx[p]:
 *   alpha = k0^2 (eps[e] - eps[eps_idx[p]]),  c = alpha / (1 - alpha diag64[p]) (FP64)
 *   FOM'  = |E[m0] + c G[m0, p] E[p]|^2     (m0 = row N + fom_monitor).
 * topk = 1: greedy rule.  With F* the largest FOM', the candidates with
 * FOM' >= F* - tau F* are tied and the lowest (pixel, eps_idx) wins; the move
 * is accepted iff F* > FOM (1 + tau), else d_out[0].pixel = -1.
 * topk = k > 1 (k <= GFO_MAX_RANK_K): the greedy rule applied k times, each
 * time to the candidates that still improve the FOM, whose pixel is not yet
 * chosen and whose Chebyshev distance to every chosen pixel is at least
 * min_spacing; unused records get pixel = -1.
 * d_out: topk device records.  A NaN/Inf score sets GFO_STATUS_NONFINITE. */
int score_candidates(const gfo_problem* prob, const gfo_state* st, uint32_t cand_mask,
                     double tau, int32_t topk, int32_t min_spacing, gfo_pick* d_out,
                     hipStream_t stream);

/* score_candidates_static - score_candidates for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same scores and the same records in d_out, bit
 * for bit, but st->work is not used (it may be NULL, as may work_bytes be 0).
 * Its scratch (N x n_eps FP64 scores and the score workgroups' summaries, at
 * most GFO_STATIC_SCRATCH_BYTES = 8 MiB: N * n_eps <= 1,047,040) lives in a
 * device array of the library, one per GPU, held until the process ends; its
 * address is taken on the first call on each device.  Allocates nothing, and
 * calls no allocating routine.  Every call on one GPU shares that GPU's
 * scratch: calls that overlap on one GPU (other streams, other threads) race
 * and must be ordered by the caller.  Returns GFO_ESCRATCH, before any launch,
 * for a problem whose scratch would not fit; GFO_EINVAL as score_candidates;
 * GFO_EHIP if the scratch address cannot be taken or a launch fails.
 * Asynchronous on `stream`. */
int score_candidates_static(const gfo_problem* prob, const gfo_state* st, uint32_t cand_mask,
                            double tau, int32_t topk, int32_t min_spacing, gfo_pick* d_out,
                            hipStream_t stream);

/* apply_flip - apply one move as a rank-1 Dyson update (paper Sec. II B,
 * eqs. form10-form14 with a one-pixel region; field by eqs. form4-form9).
 * With j = d_pick->pixel, alpha = k0^2 (eps_new - eps_j), c = alpha/(1 - alpha G_jj)
 * (FP64, from diag64):
 *   G[r, q] += c G[r, j] G[j, q]  for all rows r < R and columns q < N (in place),
 *   E[r]    += c G[r, j] E[j],     diag64[q] += c G[q, j] G[j, q] (FP64),
 *   diag64[j] = G_jj / (1 - alpha G_jj),  eps_idx[j] = eps_new, history appended.
 * The pick is read from DEVICE memory, so score -> apply needs no host round
 * trip.  A sentinel pick (pixel < 0) makes the call a no-op; a singular
 * denominator sets GFO_STATUS_SINGULAR and skips the move. */
int apply_flip(const gfo_problem* prob, gfo_state* st, const gfo_pick* d_pick,
               hipStream_t stream);

/* Deferred mode (state.delay = r > 0).  The paper's update (eq. form10) is
 * exact in any grouping, so apply_flip may postpone the design block: it
 * records c G[:, j] and G[j, :] of the CURRENT matrix (base rows plus the
 * pending terms) as pending term number s, and updates E, diag64 and the FOM
 * monitor's row of G at once.  score_candidates reads only those, so the move
 * sequence is the one of eager mode.  After r apply_flip calls since the
 * last flush, the design block and the other monitor rows are brought up to
 * date by one rank-r product on the matrix cores (FP64 for GFO_C128; for
 * GFO_C64 FP32 products, which the default flush for 17 to 128 terms computes
 * as the six leading products of three-part BF16 splits of each FP32 operand,
 * at FP32 accuracy); gfo_flush does the same on demand.  Until then those rows hold
 * their base values only.  refresh_G
 * discards pending terms (it rebuilds G from G0); apply_flips_rank_k flushes
 * first.
 * The design block G_D is symmetric at every step (reciprocity of the medium,
 * and each pending term restricted to it is c v v^T), so in deferred mode the
 * library reads its entries from the upper triangle (row <= column) only, and
 * the flushes (complex128, and every complex64 variant but "w32_3m"),
 * init_G0 and refresh_G bring only that triangle up to date; they then set
 * state.lower_stale.  In eager mode the same holds when state.lower_stale is 1
 * on entry to init_G0 or refresh_G: the rank-1 update of apply_flip then skips
 * the tiles of design rows wholly below the diagonal.  While
 * lower_stale is set, every call reads design entries from the upper
 * triangle, in eager mode too.  gfo_sync_lower copies the upper triangle into
 * the lower one for callers that read G directly. */

/* gfo_flush - bring the design block of G up to date in deferred mode (no-op
 * when nothing is pending or delay = 0).  Its lower triangle may be left out
 * of date (state.lower_stale); gfo_sync_lower completes it. */
int gfo_flush(const gfo_problem* prob, gfo_state* st, hipStream_t stream);

/* gfo_sync_lower - copy the upper triangle of the design block into its strict
 * lower triangle (G[q, p] = G[p, q] for p < q < N) when state.lower_stale is
 * set, then clear it; a no-op otherwise.  Pending deferred terms are not
 * applied (call gfo_flush first for a current matrix).  In deferred mode
 * init_G0 and refresh_G (they write the upper triangle only), the complex128
 * flush and the complex64 upper-only flush set the flag.  Asynchronous on
 * `stream`.  GFO_EINVAL for band-packed storage (no lower triangle is stored). */
int gfo_sync_lower(const gfo_problem* prob, gfo_state* st, hipStream_t stream);

/* gfo_greedy_steps - n_steps greedy moves (paper Sec. II: score every
 * one-pixel flip, take the best if it improves the FOM by more than the relative
 * band tau, apply it as the rank-1 update), with the results of n_steps calls
 * of score_candidates (topk = 1, min_spacing = 0) each followed by apply_flip
 * on its pick: the same moves, bit for bit the same state.  In deferred mode
 * (delay > 0) a move takes one kernel instead of four: every workgroup repeats
 * the pick from the previous kernel's score summaries, gathers its share of
 * the pivot row and column, applies the move to its own pixels and scores them
 * for the next move (two kernels per move on grids of more than 65,536 pixels).
 * Once the stop rule refuses a move, the remaining steps are no-ops.
 * d_picks: device array of n_steps records (the pick of each step, sentinel
 * when refused), or NULL.  n_steps >= 0; cand_mask and tau as for
 * score_candidates.  Asynchronous on `stream`. */
int gfo_greedy_steps(const gfo_problem* prob, gfo_state* st, int32_t n_steps,
                     uint32_t cand_mask, double tau, gfo_pick* d_picks, hipStream_t stream);

/* Grouped greedy steps of many resident jobs (the served form: continuous
 * batching of small jobs, whose moves are latency bound).  A job table holds,
 * per job, its geometry, buffers and workspace offsets in caller-owned device
 * memory; gfo_greedy_steps_table then runs n_steps greedy moves of every job
 * of the table with one launch per move for all of them (plus each job's own
 * flush when its term buffer is full), with the results of one
 * gfo_greedy_steps(n_steps, d_picks = NULL) call per job, bit for bit.  Jobs
 * share no memory; a job that stops (no improving move) makes no-op moves.
 * Requirements: 1 <= n_jobs <= 64, every job in deferred mode (delay > 0),
 * served by the one-kernel loop (at most 65,536 pixels), and alike in storage
 * type, term batch (delay <= 64 or not) and summary size (at most 16,384
 * pixels or not); else GFO_EINVAL. */

/* Bytes of device memory a table of n_jobs jobs needs (0 if n_jobs is out of
 * range).  Host only. */
size_t gfo_job_table_bytes(int32_t n_jobs);

/* Write the table of the jobs (probs[i], states[i]) with their candidate masks
 * and tie bands (host arrays) into d_table (256-byte aligned, at least
 * gfo_job_table_bytes(n_jobs) bytes, else GFO_ENOSPC).  The table holds the
 * jobs' device pointers: it stays valid while their buffers do, and must be
 * rebuilt when the set of jobs changes.  Exception to asynchrony: synchronises
 * `stream` once (the table is copied from host memory). */
int gfo_job_table_build(const gfo_problem* probs, const gfo_state* states, int32_t n_jobs,
                        const uint32_t* h_cand_masks, const double* h_taus, void* d_table,
                        size_t table_bytes, hipStream_t stream);

/* n_steps greedy moves of every job of a table built from these same probs and
 * states, in the same order (the host-side pending counts in states[] are kept
 * up to date as by gfo_greedy_steps).  Each job's picks go to its workspace.
 * Asynchronous on `stream`. */
int gfo_greedy_steps_table(const gfo_problem* probs, gfo_state* states, int32_t n_jobs,
                           int32_t n_steps, const void* d_table, hipStream_t stream);

/* score_regions - greedy pick among multi-pixel region moves (paper Sec. II
 * with a flipped region V of N_V = 4 pixels; Sec. IV flips 2x2-pixel pillars).
 * Square regions of side `region` (= 2) tile the design grid (ny, nx even);
 * region k = by * (nx / 2) + bx, pixels row-major inside it.  A move sets every
 * pixel of the region to one material.  Score of (k, e): B = diag(b_i) with
 * b_i = k0^2 (eps_e - eps_cur_i), x = (I - G_VV B)^-1 E_V (eqs. form6-form9),
 * FOM' = |E_m0 + G[m0, V] B x|^2 (eq. form4 at the monitor, eq. para1), solved in
 * FP64 with the FP64 diagonal; in deferred mode the in-block entries include the
 * pending terms.  Candidates: materials in cand_mask that change at least one
 * pixel.  The greedy rule and the tie band tau are those of score_candidates,
 * with (region, material) in place of (pixel, material).  Writes one record to
 * d_out (device): pixel = region index, or the sentinel.  Uses the workspace's
 * score array (then holding n_regions x n_eps region scores).  EINVAL for
 * another region side, an odd grid or more than 262144 regions. */
int score_regions(const gfo_problem* prob, const gfo_state* st, int32_t region,
                  uint32_t cand_mask, double tau, gfo_pick* d_out, hipStream_t stream);

/* gfo_region_pixels - the pixel moves of a region move (the d_out of
 * score_regions): region*region records in d_pixels (device), record i = pixel i
 * of the region with the region's material, or the sentinel where the pixel
 * already has it.  Applying them with apply_flip one after the other (any order)
 * or jointly with apply_flips_rank_k is the region update of eqs. form10-form14. */
int gfo_region_pixels(const gfo_problem* prob, const gfo_state* st, int32_t region,
                      const gfo_pick* d_region, gfo_pick* d_pixels, hipStream_t stream);

/* gfo_choose_eps_greedy - the epsilon-greedy policy of paper Sec. V: act
 * greedily with probability 1 - eps, otherwise choose at random among the top
 * improving moves.  d_top: the k records of score_candidates(topk = k,
 * min_spacing = 0) (device; improving moves first, the greedy one at index 0,
 * then sentinels).  The random numbers are inputs: the step explores iff
 * u_explore < eps, and then takes record floor(u_choice * n) of the n
 * improving ones.  Writes one record to d_out (device; the sentinel when no
 * move improves the FOM), for apply_flip.  1 <= k <= GFO_MAX_RANK_K,
 * 0 <= eps <= 1, 0 <= u < 1.  Asynchronous on `stream`. */
int gfo_choose_eps_greedy(const gfo_pick* d_top, int32_t k, double eps, double u_explore,
                          double u_choice, gfo_pick* d_out, hipStream_t stream);

/* apply_flips_rank_k - apply k moves jointly by the Woodbury form of the
 * paper's region update (eqs. form10-form14 with V = the k pixels):
 *   M = (I - B_S G[S,S])^-1 B_S  (k x k, FP64, B_S = diag(alpha)),
 *   G += G[:, S] M G[S, :],  E += G[:, S] M E[S],  diag64 updated in FP64.
 * The R x N update is a rank-k product on the matrix cores with FP32 or BF16
 * inputs (gemm_precision) and FP32 accumulation; requires GFO_C64 storage,
 * dense (GFO_EINVAL when state.packed).  In deferred mode, or with
 * state.lower_stale set, the update leaves out the blocks of design rows
 * wholly below the diagonal (about half of the design block's traffic): only
 * the upper triangle is read there.
 * Sentinel records (pixel < 0) are skipped; 1 <= k <= GFO_MAX_RANK_K. */
int apply_flips_rank_k(const gfo_problem* prob, gfo_state* st, const gfo_pick* d_picks,
                       int32_t k, int32_t gemm_precision, hipStream_t stream);

/* refresh_G - recompute G, E and diag64 of the current structure in FP64
 * from G0 and the flipped set V = {p : eps_idx[p] != background} (the
 * discretised Dyson equation, eq. form2, solved on V):
 *   G = G0 + G0[:, V] (I - B_V G0[V, V])^-1 B_V G0[V, :],
 *   E = Einc + G0[:, V] (I - B_V G0[V, V])^-1 B_V Einc[V],
 * then rounds G and E once to the storage type.  Removes the rounding drift
 * of repeated rank-1 updates, and discards pending deferred terms (the
 * rebuilt G includes every accepted move).  Requires init_G0 on this workspace
 * and |V| <= kmax.  |V| is counted first: with |V| > kmax the call returns
 * GFO_ERANGE and sets GFO_STATUS_REFRESH_OVERFLOW, and nothing else changes
 * (G, E, diag64, the pending deferred terms and state.pending_calls are left
 * as they were).  The design block is computed on and above its diagonal (it
 * is symmetric); in deferred mode, or with state.lower_stale set, only that
 * triangle is written (state.lower_stale set), otherwise the lower triangle is
 * written as its mirror.  Exception to asynchrony:
 * synchronises `stream` once, to read |V|, before any of the rebuild is
 * enqueued. */
int refresh_G(const gfo_problem* prob, gfo_state* st, hipStream_t stream);

/* Autotuner hooks for the streaming rank-1 kernel of apply_flip: the kernel
 * exists in several tile shapes (rows per workgroup x rows in flight, plain or
 * non-temporal memory operations), all computing bit-identical results.
 * Selection is process-wide per storage type; host only. */
int gfo_k1_variant_count(int32_t dtype);
const char* gfo_k1_variant_name(int32_t dtype, int32_t idx);   /* NULL if out of range */
int gfo_k1_set_variant(int32_t dtype, int32_t idx);           /* GFO_EINVAL if out of range */
int gfo_k1_get_variant(int32_t dtype);

/* Autotuner hooks for the matrix-core update of apply_flips_rank_k: tile and
 * epilogue variants of the same rank-k product (the streaming variants agree
 * with each other bit for bit; the accumulating one, "acc64", differs from
 * them by FP32 rounding).  Selection is process-wide; host only. */
int gfo_rk_variant_count(void);
const char* gfo_rk_variant_name(int32_t idx);                 /* NULL if out of range */
int gfo_rk_set_variant(int32_t idx);                          /* GFO_EINVAL if out of range */
int gfo_rk_get_variant(void);

/* Autotuner hooks for the complex64 deferred-mode flush: tile variants of the
 * same rank-r matrix-core product (bit-identical results are not guaranteed
 * across variants: the FP32 summation order, and for "up_bandseg_s3" the
 * product's arithmetic, differ).  Host only. */
int gfo_flush_variant_count(void);
const char* gfo_flush_variant_name(int32_t idx);              /* NULL if out of range */
int gfo_flush_set_variant(int32_t idx);                       /* GFO_EINVAL if out of range */
int gfo_flush_get_variant(void);

/* Test and benchmark hook for gfo_greedy_steps in deferred mode: form 0
 * (default) runs one kernel per move on grids of up to 65,536 pixels and two
 * kernels per move above; form 1 runs two kernels per move on every grid.  Both
 * forms make the same moves and leave bit for bit the same state.
 * Process-wide; host only. */
int gfo_loop_set_form(int32_t form);                          /* GFO_EINVAL unless 0 or 1 */
int gfo_loop_get_form(void);

/* Timing hook: the next G update (on any stream) records `before` on its
 * stream immediately before its G-update kernel (the streaming rank-1 kernel
 * of apply_flip, the matrix-core rank-k kernels of apply_flips_rank_k, or the
 * design-block kernel of a deferred-mode flush) and `after` immediately after
 * it, then forgets both events.  Lets a caller time that
 * kernel alone with hipEventElapsedTime.  Both NULL cancels a pending pair.
 * Host only; one pending pair per process. */
int gfo_time_next_k1(hipEvent_t before, hipEvent_t after);

#ifdef __cplusplus
}
#endif
#endif /* GFO_H */
