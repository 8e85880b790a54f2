// Internal definitions shared by the libgfo HIP sources: the kernel parameter
// block, FP64 complex helpers, storage-type traits and the workspace layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/gfo.h"

namespace gfo {

// Keeps e as the calling thread's last failed HIP result (read back through
// gfo_last_hip_error) when it is not hipSuccess; returns e.
hipError_t note_hip(hipError_t e);
// Drops a HIP error left by calls made before the entry point (called first
// in every entry point that launches kernels).
void discard_stale_hip();
// Records ev on s when ev is set (the autotuner's timing events).
inline hipError_t record_event(hipEvent_t ev, hipStream_t s) {
  return ev ? hipEventRecord(ev, s) : hipSuccess;
}

// Geometry and material data passed by value to every kernel.
struct Geo {
  int ny, nx, nmon, N, R;
  int64_t ld;
  double k0, k0sq, h;
  double eps[GFO_MAX_EPS];
  int n_eps, bg_idx, m0;
  int dtype;
  // 1: entries of the design block are read from its upper triangle (row <=
  // column).  The block is symmetric (reciprocity of the medium), and in
  // deferred mode a flush may bring only the upper triangle up to date.
  int upper;
  // 1: band-packed storage of the design block's upper triangle (see g_off);
  // implies upper.  mon_base: offset of the first monitor row.
  int packed;
  int64_t mon_base;
};

// Band-packed storage: design rows in bands of 64; the rows of band b store the
// columns [64 b, ld) only (the tiles on and above the diagonal), band b starts
// at 64 (b ld - 32 b (b - 1)) and its rows are ld - 64 b apart; every row
// starts on a 64-entry boundary.  The monitor rows follow, ld apart.  Dense
// storage: row r at r ld.
__host__ __device__ __forceinline__ int64_t g_band_start(int packed, int64_t ld, int64_t b) {
  return packed ? 64 * (b * ld - 32 * b * (b - 1)) : 64 * b * ld;
}
__host__ __device__ __forceinline__ int64_t g_band_stride(int packed, int64_t ld, int64_t b) {
  return packed ? ld - 64 * b : ld;
}
// Entries of G for a problem of N design pixels: packed, the design bands and
// the monitor rows; dense, R x ld.
__host__ __device__ __forceinline__ int64_t g_elems(int packed, int64_t N, int64_t nmon, int64_t ld) {
  return packed ? g_band_start(1, ld, (N + 63) / 64) + nmon * ld : (N + nmon) * ld;
}

// Offset of entry (r, c) of G as stored (packed: design entries need
// c >= 64 (r / 64)).
__host__ __device__ __forceinline__ int64_t g_off(const Geo& g, int64_t r, int64_t c) {
  if (!g.packed) return r * g.ld + c;
  if (r >= g.N) return g.mon_base + (r - g.N) * g.ld + c;
  const int64_t b = r >> 6;
  return g_band_start(1, g.ld, b) + (r & 63) * (g.ld - 64 * b) + (c - 64 * b);
}

// Offset of entry (p, q) of G; design-block entries (p, q < N) come from the
// upper triangle when g.upper.
__device__ __forceinline__ int64_t g_at(const Geo& g, int64_t p, int64_t q) {
  return g.upper && p > q && p < g.N ? g_off(g, q, p) : g_off(g, p, q);
}

// ------------------------------------------------------------------ complex FP64
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// real / complex
__device__ __forceinline__ double2 rdiv(double a, double2 d) {
  double n = d.x * d.x + d.y * d.y;
  return make_double2(a * d.x / n, -a * d.y / n);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------------ storage traits
template <typename T> struct St;
template <> struct St<float2> {
  __device__ __forceinline__ static double2 to_d(float2 v) { return make_double2((double)v.x, (double)v.y); }
  __device__ __forceinline__ static float2 from_d(double2 v) { return make_float2((float)v.x, (float)v.y); }
};
template <> struct St<double2> {
  __device__ __forceinline__ static double2 to_d(double2 v) { return v; }
  __device__ __forceinline__ static double2 from_d(double2 v) { return v; }
};

// ------------------------------------------------------------------ reductions
// Wave-wide max and min over all 64 lanes (every lane active), with the ROCm
// device library's wave reductions (cross-lane data-parallel moves instead of
// LDS permutes).  Exact operations, so the result does not depend on the order.
extern "C" __device__ __attribute__((const)) double __ockl_wfred_max_f64(double);
extern "C" __device__ __attribute__((const)) int __ockl_wfred_min_i32(int);
__device__ __forceinline__ double wave_max(double v) { return __ockl_wfred_max_f64(v); }
__device__ __forceinline__ int wave_min(int v) { return __ockl_wfred_min_i32(v); }
// block-wide max; all threads get the result. `sh` holds blockDim/64 doubles.
__device__ inline double block_max(double v, double* sh) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = -INFINITY;
  for (int i = 0; i < nw; ++i) r = fmax(r, sh[i]);
  return r;
}
__device__ inline int block_min(int v, int* sh) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_min(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  int r = 0x7fffffff;
  for (int i = 0; i < nw; ++i) r = min(r, sh[i]);
  return r;
}

// Snapshot of the accepted move, written before G is modified.
struct Snap {
  int32_t j;          // pixel, -1 = no move
  int32_t e_new;
  int32_t slot;       // deferred mode: index of this move's pending term
  int32_t pad1;       // deferred mode: 1 = singular denominator, move refused
  double alpha;
  double pad2;
  double2 c;          // alpha / (1 - alpha G_jj)
  double2 Ej;         // E[j] before the move
  double2 dj;         // G_jj before the move (FP64)
  // one-kernel greedy loop: the pivot's values after the move (E[j] and
  // G[N+m0, j] in the storage type's values, the FP64 diagonal), written to
  // memory by the next kernel, and the term count after the move
  double2 Ej_new, dj_new, gm0_new;
  int32_t cnt_after, pad3, pad4, pad5;
};

constexpr int kScoreThreads = 256;
constexpr int kScoreMaxBlocks = 1024;
// 16-byte units per index of the split-product flush's operands: 12 per 16
// pending terms, up to GFO_MAX_DELAY terms.
constexpr int kSplitUnits = 12 * (GFO_MAX_DELAY / 16);
constexpr int kSelectThreads = 1024;

// ------------------------------------------------------------------ workspace layout
struct Layout {
  size_t table;     // ny*nx double2: G0 over non-negative pixel offsets
  size_t mon_xy;    // 2*nmon double
  size_t scores;    // N*n_eps double
  size_t partial;   // kScoreMaxBlocks double: best score of each score workgroup
  size_t pfirst;    // kScoreMaxBlocks int32: lowest index within the tie band of that best
  size_t picks;     // GFO_MAX_RANK_K gfo_pick (internal rank-k scratch)
  size_t snap;      // Snap
  size_t cu;        // R x 16 B: c * G[:, j] (storage type)
  size_t v;         // ld x 16 B: G[j, :] (storage type), zero padded to ld
  size_t emon;      // nmon x 16 B: E at the monitors after the last gathered move
  // second buffers of the one-kernel greedy loop (kernel t reads one set and
  // writes the other)
  size_t snap2, emon2, scores2, partial2, pfirst2;
  // rank-k
  size_t rk_S;      // header of the accepted set (pixels, contrasts, M E[S])
  size_t rk_M;      // K x K double2 (FP64 Woodbury core)
  size_t rk_U64;    // R x K double2: G[:, S] in FP64
  size_t rk_A;      // R x 2K float  A operand [Re U | Im U] (U = G[:, S])
  size_t rk_B;      // 2 x 2K x ld float: B operands for the re and im outputs
  size_t rk_Abf;    // R x 2K bf16
  size_t rk_Bbf;    // 2 x 2K x ld bf16
  // deferred rank-1 terms (GFO_MAX_DELAY slots)
  size_t dl_hdr;    // int32 count of pending terms
  size_t dl_CUs;    // GFO_MAX_DELAY x R x 16 B: c * G[:, j] of each pending move, slot-major
  size_t dl_Vs;     // GFO_MAX_DELAY x ld x 16 B: G[j, :] of each pending move, slot-major
  // refresh
  // (kp = kmax rounded up to a multiple of 4)
  size_t rf_V;      // N + 1 int32: flipped list, then its length
  size_t rf_U;      // R x kp double2: G0[:, V]
  size_t rf_A;      // 2 kp^2 double2: two kp x kp buffers of the in-place Gauss-Jordan inverse
                    // of diag(1/alpha) - G0[V,V], then M
  size_t rf_piv;    // 16 kp + 64 bytes: the steps' pivot candidates, the pivots, the used rows
  size_t rf_Z;      // R x kp double2: G0[:, V] M; before it, the blocked inverse's panel buffers
  size_t rf_x;      // kp double2: M Einc[V]
  // split-product flush (complex64 storage only): the pending terms as BF16
  // parts, kSplitUnits units of 16 bytes per row (R rows of CU) and per column
  // (ld columns of V)
  size_t dl_split;
  size_t total;
};

// Scores of pixel p for every material (eqs. form4-form9 at the FOM monitor):
// F = |E_m0 + c G[m0, p] E_p|^2 with c = alpha / (1 - alpha G_pp) in FP64; -inf
// for non-candidates and the current material.  Writes them to `scores` and to
// F[0 .. n_eps) (a register array: the loop is unrolled over GFO_MAX_EPS), returns
// the largest and sets *bad on a non-finite one.
__device__ inline double score_pixel(const Geo& g, int p, int cur, double2 d, double2 gE,
                                     double2 Em0, uint32_t mask, double* __restrict__ scores,
                                     bool* bad, double (&F)[GFO_MAX_EPS]) {
  double best = -INFINITY;
#pragma unroll
  for (int e = 0; e < GFO_MAX_EPS; ++e) {
    if (e < g.n_eps) {
      double Fe = -INFINITY;
      if (((mask >> e) & 1u) && e != cur) {
        const double a = g.k0sq * (g.eps[e] - g.eps[cur]);
        const double2 c = rdiv(a, make_double2(1.0 - a * d.x, -a * d.y));   // FP64 denominator
        const double2 En = cadd(Em0, cmul(c, gE));
        Fe = cabs2(En);
        if (!isfinite(Fe)) {
          *bad = true;
          Fe = -INFINITY;
        }
        best = fmax(best, Fe);
      }
      F[e] = Fe;
      scores[(int64_t)p * g.n_eps + e] = Fe;
    }
  }
  return best;
}

// Relative tie band of the greedy rule: scores within tau of the best, m.
__device__ __forceinline__ double tie_threshold(double m, double tau) { return m - tau * m; }

// Lowest (pixel, material) index of pixel p whose score reaches thr, else INT_MAX.
__device__ inline int first_at_least(const Geo& g, int p, const double (&F)[GFO_MAX_EPS],
                                     double thr) {
  int f = 0x7fffffff;
#pragma unroll
  for (int e = GFO_MAX_EPS - 1; e >= 0; --e)
    if (e < g.n_eps && F[e] >= thr) f = p * g.n_eps + e;
  return f;
}

// End of a score workgroup that scored one pixel per thread: partial[b] = its
// best score, pfirst[b] = the lowest index whose score is within the tie band of
// that best (INT_MAX if no candidate, or when has_F is false: pixels of a
// thread not all in F).  All threads of the workgroup must call it.
__device__ inline void score_block_end(const Geo& g, double best, int p, bool has_F,
                                       const double (&F)[GFO_MAX_EPS], double tau,
                                       double* __restrict__ partial, int* __restrict__ pfirst,
                                       int nblk, double* shd, int* shi) {
  const double bb = block_max(best, shd);
  int f = 0x7fffffff;
  if (has_F && p < g.N && bb > -INFINITY) f = first_at_least(g, p, F, tie_threshold(bb, tau));
  f = block_min(f, shi);
  if (threadIdx.x == 0 && (int)blockIdx.x < nblk) {
    partial[blockIdx.x] = bb;
    pfirst[blockIdx.x] = f;
  }
}

// The greedy pick over scores written one pixel per thread by workgroups of
// kScoreThreads (workgroup b covered pixels [b * kScoreThreads, ...) and left
// partial[b] and pfirst[b], score_block_end): accept the best score F* only if
// F* > fom (1 + tau); the winner is the lowest (pixel, material) index whose
// score is within the relative band tau of F*.  It lies in the lowest workgroup
// whose maximum reaches the band (that maximum itself qualifies); if that
// workgroup holds F*, pfirst is the winner, otherwise (a near-tie across
// workgroups) its scores are scanned.  Every thread of the calling workgroup
// gets the pick.
__device__ inline gfo_pick greedy_pick_block(const Geo& g, double fom,
                                             const double* __restrict__ scores,
                                             const double* __restrict__ partial,
                                             const int* __restrict__ pfirst, int nblk, double tau,
                                             double* shd, int* shi) {
  gfo_pick pk;
  pk.pixel = -1;
  pk.eps_idx = -1;
  pk.fom_new = fom;
  pk.dfom = 0.0;
  double m = -INFINITY;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) m = fmax(m, partial[i]);
  m = block_max(m, shd);
  if (!(m > fom * (1.0 + tau))) return pk;
  const double thr = tie_threshold(m, tau);
  int bq = 0x7fffffff;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    if (partial[i] >= thr) {
      bq = i;
      break;
    }
  }
  bq = block_min(bq, shi);
  int first = 0x7fffffff;
  const int pf = pfirst[bq];
  if (partial[bq] == m && pf != 0x7fffffff) {
    first = pf;
  } else {
    const int total = g.N * g.n_eps, span = kScoreThreads * g.n_eps;
    const int lo = bq * span, hi = min(lo + span, total);
    int f = 0x7fffffff;
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      if (scores[i] >= thr) {
        f = i;
        break;
      }
    }
    first = block_min(f, shi);
  }
  if (first == 0x7fffffff) return pk;
  pk.pixel = first / g.n_eps;
  pk.eps_idx = first - pk.pixel * g.n_eps;
  pk.fom_new = scores[first];
  pk.dfom = pk.fom_new - fom;
  return pk;
}

// The same pick taken by each wave on its own (no LDS, no barrier), in two
// steps so that a caller can put other loads in flight between them:
// pick_wave_load reads the workgroup summaries (lane l holds partial[l + 64 k]
// and pfirst[l + 64 k]), pick_wave_take reduces them with cross-lane
// operations and takes the winning workgroup's entries from the lane that
// holds them, so the pick costs one round trip to memory (plus a scan of one
// workgroup's scores in a near-tie across workgroups).  Same decisions as
// greedy_pick_block (exact max and min).  PPL summaries per lane: up to 64 PPL
// workgroup summaries (the caller picks the smallest that covers its grid, as
// the reductions walk every register).
constexpr int kPickPerLane = kScoreMaxBlocks / 64;

template <int PPL = kPickPerLane>
struct PickPre {
  double pv[PPL];
  int pf[PPL];
};

template <int PPL>
__device__ __forceinline__ void pick_wave_load(const double* __restrict__ partial,
                                               const int* __restrict__ pfirst, int nblk,
                                               PickPre<PPL>& pp) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int i = lane + 64 * k;
    pp.pv[k] = -INFINITY;
    pp.pf[k] = 0x7fffffff;
    if (i < nblk) {
      pp.pv[k] = partial[i];
      pp.pf[k] = pfirst[i];
    }
  }
}

// with_score = false leaves fom_new and dfom of an accepted pick unset (the
// caller reads scores[pixel * n_eps + eps_idx] where it needs them).
template <int PPL>
__device__ __forceinline__ gfo_pick pick_wave_take(const Geo& g, double fom, const PickPre<PPL>& pp,
                                                   const double* __restrict__ scores, double tau,
                                                   bool with_score = true,
                                                   int bpix = kScoreThreads) {
  gfo_pick pk;
  pk.pixel = -1;
  pk.eps_idx = -1;
  pk.fom_new = fom;
  pk.dfom = 0.0;
  const int lane = threadIdx.x & 63;
  double m = -INFINITY;
#pragma unroll
  for (int k = 0; k < PPL; ++k) m = fmax(m, pp.pv[k]);
  m = wave_max(m);
  if (!(m > fom * (1.0 + tau))) return pk;
  const double thr = tie_threshold(m, tau);
  int bq = 0x7fffffff;
#pragma unroll
  for (int k = PPL - 1; k >= 0; --k)
    if (pp.pv[k] >= thr) bq = lane + 64 * k;
  bq = __builtin_amdgcn_readfirstlane(wave_min(bq));
  // workgroup bq's summary, from lane bq % 64, register bq / 64
  const int kb = bq >> 6, lb = bq & 63;
  double pvb = -INFINITY;
  int pfb = 0x7fffffff;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    if (k == kb) {
      pvb = pp.pv[k];
      pfb = pp.pf[k];
    }
  }
  const int pf = __builtin_amdgcn_readlane(pfb, lb);
  const double pb = __builtin_bit_cast(
      double, ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(__builtin_bit_cast(uint64_t, pvb) >> 32), lb)
               << 32) |
                  (uint32_t)__builtin_amdgcn_readlane((int)__builtin_bit_cast(uint64_t, pvb), lb));
  int first = 0x7fffffff;
  if (pb == m && pf != 0x7fffffff) {
    first = pf;
  } else {
    const int total = g.N * g.n_eps, span = bpix * g.n_eps;
    const int lo = bq * span, hi = min(lo + span, total);
    int f = 0x7fffffff;
    for (int i = lo + lane; i < hi; i += 64) {
      if (scores[i] >= thr) {
        f = i;
        break;
      }
    }
    first = wave_min(f);
  }
  first = __builtin_amdgcn_readfirstlane(first);
  if (first == 0x7fffffff) return pk;
  pk.pixel = first / g.n_eps;
  pk.eps_idx = first - pk.pixel * g.n_eps;
  if (with_score) {
    pk.fom_new = scores[first];
    pk.dfom = pk.fom_new - fom;
  }
  return pk;
}

Layout make_layout(const gfo_problem* p, int64_t ld, int32_t kmax);
Geo make_geo(const gfo_problem* p, int64_t ld);
// make_geo for a job: upper = deferred mode or an out-of-date lower triangle
Geo make_geo(const gfo_problem* p, const gfo_state* st);
int validate_problem(const gfo_problem* p);
int find_bg(const gfo_problem* p);

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------------ launchers
hipError_t launch_init(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s);
hipError_t launch_score(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                        double tau, int topk, int spacing, gfo_pick* out, hipStream_t s);
// Scratch of score_candidates: N x n_eps scores, then per score workgroup its
// best score and the lowest index within the tie band of that best.
struct ScoreBufs {
  double* scores;
  double* partial;
  int* pfirst;
};
// workgroups of the score kernel (one pixel per thread, at most kScoreMaxBlocks)
inline int score_blocks(const Geo& g) {
  const int n = (g.N + kScoreThreads - 1) / kScoreThreads;
  return n < kScoreMaxBlocks ? n : kScoreMaxBlocks;
}
hipError_t launch_score_into(const Geo& g, const gfo_state* st, const ScoreBufs& b, uint32_t mask,
                             double tau, int topk, int spacing, gfo_pick* out, hipStream_t s);
int validate_state_fields(const gfo_problem* p, const gfo_state* st);
int validate_job(const gfo_problem* p, const gfo_state* st, Layout* L);
hipError_t launch_apply(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                        hipStream_t s);
hipError_t launch_rank_k(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* picks,
                         int k, int precision, hipStream_t s);
// refresh_G in two parts: the flipped list and its length k (synchronises the
// stream), then the rebuild for that list (k <= kmax)
int launch_refresh_count(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s, int32_t* k);
hipError_t launch_refresh_overflow(gfo_state* st, hipStream_t s);
int launch_refresh(const Geo& g, gfo_state* st, const Layout& L, int32_t k, hipStream_t s);
hipError_t launch_flush(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s);
hipError_t launch_sync_lower(const Geo& g, gfo_state* st, hipStream_t s);
template <typename T>
hipError_t launch_apply_deferred(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                                 hipStream_t s);
hipError_t launch_zgemm_update_f64(const Geo& g, const int32_t* count, const double2* CU,
                                   const double2* V, double2* G, hipStream_t s);
hipError_t launch_dl_reset(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s);
int region_side();
hipError_t launch_score_regions(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                                double tau, gfo_pick* out, hipStream_t s);
hipError_t launch_region_pixels(const Geo& g, const gfo_state* st, const gfo_pick* region,
                                gfo_pick* out, hipStream_t s);
hipError_t launch_choose_eps_greedy(const gfo_pick* top, int k, double eps, double u_explore,
                                    double u_choice, gfo_pick* out, hipStream_t s);
// one-kernel greedy loop (deferred mode)
bool one_kernel_loop(const Geo& g);
template <typename T>
hipError_t launch_move_scores(const Geo& g, gfo_state* st, const Layout& L, uint32_t mask,
                              double tau, hipStream_t s);
template <typename T>
hipError_t launch_move(const Geo& g, gfo_state* st, const Layout& L, int t, int flushed,
                       uint32_t mask, double tau, gfo_pick* pick_out, hipStream_t s);
template <typename T>
hipError_t launch_move_finish(const Geo& g, gfo_state* st, const Layout& L, int t, hipStream_t s);
template <typename T>
hipError_t launch_fused_move(const Geo& g, gfo_state* st, const Layout& L, int apply_prev,
                             uint32_t mask, double tau, gfo_pick* pick_out, bool flush_between,
                             hipStream_t s);
template <typename T>
hipError_t launch_fused_finish(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s);

// ------------------------------------------------------------------ XCD tile order
// Tiles of an upper-triangle flush (nb x nb design tiles on and above the
// diagonal, then nmb rows of nbx monitor tiles), numbered so that workgroup b
// (the dispatcher sends workgroup b to XCD b % 8) takes tiles of the column
// blocks bx with bx % 8 == b % 8 only: XCD x walks its own tiles row by row
// (triangle rows first, then monitor rows), so its L2 holds just the operand
// panels of its eighth of the columns, while the eight XCDs sweep the same rows
// of G together.  Returns false when workgroup b has no tile (the grid is 8
// times the largest per-XCD count).
__host__ __device__ inline int xcd_cols_below(int n, int x) {   // #{c < n : c % 8 == x}
  return n > x ? (n - x + 7) / 8 : 0;
}
__host__ __device__ inline int xcd_tri_before(int by, int nb, int x) {
  // XCD x's triangle tiles in rows [0, by): sum over rows i < by of
  // #{c in [i, nb) : c % 8 == x} = by * cols(nb) - sum_{i < by} cols(i)
  const int m = by - 1 - x;
  int lower = 0;
  if (m > 0) {
    const int q = m / 8, r = m % 8;
    lower = 4 * q * (q + 1) + r * (q + 1);
  }
  return by * xcd_cols_below(nb, x) - lower;
}
__host__ __device__ inline int xcd_tile_count(int nb, int nbx, int nmb, int x) {
  return xcd_tri_before(nb, nb, x) + nmb * xcd_cols_below(nbx, x);
}
__host__ __device__ inline bool xcd_tile(int b, int nb, int nbx, int nmb, int* by, int* bx,
                                         bool* mon) {
  const int x = b & 7, local = b >> 3;
  const int ntri = xcd_tri_before(nb, nb, x);
  if (local < ntri) {
    int lo = 0, hi = nb - 1;                 // the last row whose start is <= local
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (xcd_tri_before(mid, nb, x) <= local) lo = mid; else hi = mid - 1;
    }
    const int k = local - xcd_tri_before(lo, nb, x);
    const int c0 = lo + ((x - lo % 8) + 8) % 8;   // first column >= lo with c % 8 == x
    *by = lo;
    *bx = c0 + 8 * k;
    *mon = false;
    return *bx < nb;
  }
  const int per = xcd_cols_below(nbx, x);
  if (per == 0) return false;
  const int l2 = local - ntri, mby = l2 / per;
  if (mby >= nmb) return false;
  *by = mby;
  *bx = x + 8 * (l2 - mby * per);
  *mon = true;
  return *bx < nbx;
}

// ------------------------------------------------------------------ job table
// One entry per job of a grouped launch (gfo_greedy_steps_table): its geometry,
// its buffers and the workspace offsets the one-kernel loop uses, and the
// workgroup counts of its kernels.  Built on the host, read by the table
// kernels (workgroup (x, y) works for job y as workgroup x of its own launch).
struct JobEntry {
  Geo g;
  void* G;
  void* E;
  double2* diag64;
  uint8_t* eps_idx;
  int32_t* flips;
  int32_t* n_flips;
  int32_t* status;
  char* work;
  int64_t snap, snap2, emon, emon2, scores, scores2, partial, partial2, pfirst, pfirst2;
  int64_t cu, v, dl_hdr, dl_CUs, dl_Vs, picks;
  double tau;
  uint32_t mask;
  int32_t flip_cap;
  int32_t n_score_wg;   // workgroups of the scoring kernel (kScoreThreads indices each)
  int32_t n_move_wg;    // workgroups of the move kernel (kGatherElems elements each)
  int32_t n_finish_wg;  // workgroups of the finishing kernel
  int32_t nblk0;        // score summaries of the scoring kernel (kScoreThreads pixels each)
  int32_t nblkg;        // score summaries of the move kernel (kGatherElems pixels each)
  int32_t pad[3];
};
JobEntry make_job_entry(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                        double tau);
// the grouped kernels: every job of the table, one launch each
template <typename T>
hipError_t launch_table_scores(const JobEntry* tab, int n_jobs, int max_wg, hipStream_t s);
template <typename T>
hipError_t launch_table_move(const JobEntry* tab, int n_jobs, int max_wg, int t, uint64_t flushed,
                             bool small, int batch, hipStream_t s);
template <typename T>
hipError_t launch_table_finish(const JobEntry* tab, int n_jobs, int max_wg, int t, hipStream_t s);
int gather_move_workgroups(const Geo& g);
bool move_small_grid(const Geo& g);

// K1 variant selection (autotuner); returns number of variants
int k1_variant_count(int dtype);
const char* k1_variant_name(int dtype, int idx);
int k1_set_variant(int dtype, int idx);
int k1_get_variant(int dtype);
void k1_time_next(hipEvent_t before, hipEvent_t after);
void k1_take_timing(hipEvent_t* before, hipEvent_t* after);   // consumes the pending pair
// the streaming rank-1 update of G with the selected tile variant (timed if requested)
hipError_t launch_rank1(const Geo& g, const Snap* snap, const void* cu, const void* v, void* G,
                        hipStream_t s);
int rk_variant_count();
const char* rk_variant_name(int idx);
int rk_set_variant(int idx);
int rk_get_variant();
int flush_variant_count();
const char* flush_variant_name(int idx);
int flush_set_variant(int idx);
int flush_get_variant();

// Updates of the design block's upper triangle alone launch only the workgroups
// that write something (a workgroup that returned at once would still take a
// dispatch slot).  Row groups of H rows, column groups of W columns (H and W
// powers of two): a row group y below nskip = N / H (wholly in design rows)
// keeps the column groups [lo(y), ncg), lo(y) = floor(y H / W), the groups that
// reach column y H or beyond; later row groups keep every column group.  With
// nskip = 0 this is the plain row-major mapping.
__host__ __device__ inline int64_t ut_lo_sum(int64_t y, int H, int W) {   // sum of lo(i), i < y
  if (H >= W) return (int64_t)(H / W) * y * (y - 1) / 2;
  const int64_t d = W / H, q = y / d;
  return d * q * (q - 1) / 2 + q * (y - q * d);
}
__host__ __device__ inline int64_t ut_first(int64_t y, int ncg, int H, int W) {  // launch index of row group y
  return y * ncg - ut_lo_sum(y, H, W);
}
__host__ inline int64_t ut_group_count(int nrg, int ncg, int nskip, int H, int W) {
  return ut_first(nskip, ncg, H, W) + (int64_t)(nrg - nskip) * ncg;
}
__device__ __forceinline__ void ut_group(int64_t t, int ncg, int nskip, int H, int W, int& rg, int& cg) {
  const int64_t t1 = ut_first(nskip, ncg, H, W);
  if (t >= t1) {
    t -= t1;
    rg = nskip + (int)(t / ncg);
    cg = (int)(t % ncg);
    return;
  }
  int lo = 0, hi = nskip - 1;   // the last row group whose first index is <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ut_first(mid, ncg, H, W) <= t) lo = mid;
    else hi = mid - 1;
  }
  rg = lo;
  cg = (int)((int64_t)lo * H / W + (t - ut_first(lo, ncg, H, W)));
}

}  // namespace gfo
