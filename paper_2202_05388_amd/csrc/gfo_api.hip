// Host side of the C ABI declared in include/gfo.h: argument validation,
// workspace layout and dispatch to the kernel launchers.
#include "gfo_internal.hpp"

#include <math.h>
#include <string.h>

#include <atomic>

namespace gfo {

// Form of the deferred-mode greedy loop (gfo_loop_set_form): 0 automatic, 1
// two kernels per move.
static std::atomic<int> g_loop_form{0};

int find_bg(const gfo_problem* p) {
  for (int i = 0; i < p->n_eps; ++i)
    if (p->h_eps_table[i] == p->eps_bg) return i;
  return -1;
}

int validate_problem(const gfo_problem* p) {
  if (!p) return GFO_EINVAL;
  if (p->ny < 1 || p->nx < 1 || p->n_mon < 1) return GFO_EINVAL;
  if (p->dtype != GFO_C64 && p->dtype != GFO_C128) return GFO_EINVAL;
  if (!(p->wavelength > 0.0) || !(p->pitch > 0.0)) return GFO_EINVAL;
  if (p->n_eps < 2 || p->n_eps > GFO_MAX_EPS || !p->h_eps_table || !p->h_mon_xy) return GFO_EINVAL;
  if (p->fom_monitor < 0 || p->fom_monitor >= p->n_mon) return GFO_EINVAL;
  const int64_t N = (int64_t)p->ny * p->nx;
  if (N * p->n_eps >= (int64_t)1 << 31 || N + p->n_mon >= (int64_t)1 << 31) return GFO_EINVAL;
  for (int i = 0; i < p->n_eps; ++i)
    if (!isfinite(p->h_eps_table[i])) return GFO_EINVAL;
  for (int i = 0; i < 2 * p->n_mon; ++i)
    if (!isfinite(p->h_mon_xy[i])) return GFO_EINVAL;
  if (find_bg(p) < 0) return GFO_EINVAL;
  return GFO_OK;
}

Geo make_geo(const gfo_problem* p, int64_t ld) {
  Geo g = {};
  g.ny = p->ny;
  g.nx = p->nx;
  g.nmon = p->n_mon;
  g.N = p->ny * p->nx;
  g.R = g.N + p->n_mon;
  g.ld = ld;
  g.k0 = 2.0 * 3.14159265358979323846 / p->wavelength;
  g.k0sq = g.k0 * g.k0;
  g.h = p->pitch;
  for (int i = 0; i < p->n_eps; ++i) g.eps[i] = p->h_eps_table[i];
  g.n_eps = p->n_eps;
  g.bg_idx = find_bg(p);
  g.m0 = p->fom_monitor;
  g.dtype = p->dtype;
  g.mon_base = (int64_t)g.N * ld;
  return g;
}

Geo make_geo(const gfo_problem* p, const gfo_state* st) {
  Geo g = make_geo(p, st->ldG);
  g.packed = st->packed;
  g.upper = st->packed || st->delay > 0 || st->lower_stale ? 1 : 0;
  g.mon_base = g_elems(g.packed, g.N, 0, g.ld);
  return g;
}

Layout make_layout(const gfo_problem* p, int64_t ld, int32_t kmax) {
  const size_t N = (size_t)p->ny * p->nx, R = N + p->n_mon, K = GFO_MAX_RANK_K;
  const size_t k = kmax > 0 ? ((size_t)kmax + 3) / 4 * 4 : 0;   // padded to the MFMA k-step
  Layout L = {};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.table = take(N * 16);
  L.mon_xy = take((size_t)p->n_mon * 16);
  L.scores = take(N * p->n_eps * 8);
  L.partial = take(kScoreMaxBlocks * 8);
  L.pfirst = take(kScoreMaxBlocks * 4);
  L.picks = take(K * sizeof(gfo_pick));
  L.snap = take(sizeof(Snap));
  L.cu = take(R * 16);
  L.v = take((size_t)ld * 16);
  L.emon = take((size_t)p->n_mon * 16);
  L.snap2 = take(sizeof(Snap));
  L.emon2 = take((size_t)p->n_mon * 16);
  L.scores2 = take(N * p->n_eps * 8);
  L.partial2 = take(kScoreMaxBlocks * 8);
  L.pfirst2 = take(kScoreMaxBlocks * 4);
  L.rk_S = take(4096);
  L.rk_M = take(K * K * 16);
  L.rk_U64 = take(R * K * 16);
  L.rk_A = take(R * 2 * K * 4);
  L.rk_B = take(2 * 2 * K * (size_t)ld * 4);
  L.rk_Abf = take(R * 2 * K * 2);
  L.rk_Bbf = take(2 * 2 * K * (size_t)ld * 2);
  L.dl_hdr = take(256);
  L.dl_CUs = take((size_t)GFO_MAX_DELAY * R * 16);
  L.dl_Vs = take((size_t)GFO_MAX_DELAY * (size_t)ld * 16);
  L.rf_V = take((N + 64) * 4);
  L.rf_U = take(R * k * 16);
  L.rf_A = take(2 * k * k * 16);
  L.rf_piv = take(k * 16 + 64);
  L.rf_Z = take(R * k * 16);
  L.rf_x = take(k * 16 + 64);
  L.dl_split = p->dtype == GFO_C64 ? take((size_t)kSplitUnits * (R + (size_t)ld) * 16) : 0;
  L.total = o;
  return L;
}

static int64_t min_ld(const gfo_problem* p) {
  const int64_t N = (int64_t)p->ny * p->nx;
  return (N + 63) / 64 * 64;
}

// Every field of a job's state except the workspace.
int validate_state_fields(const gfo_problem* p, const gfo_state* st) {
  if (!st || !st->G || !st->E || !st->diag64 || !st->eps_idx || !st->n_flips || !st->status)
    return GFO_EINVAL;
  if (st->flip_cap < 0 || (st->flip_cap > 0 && !st->flips) || st->kmax < 0) return GFO_EINVAL;
  if (st->delay < 0 || st->delay > GFO_MAX_DELAY || st->pending_calls < 0) return GFO_EINVAL;
  if (st->lower_stale != 0 && st->lower_stale != 1) return GFO_EINVAL;
  // band-packed storage holds the upper triangle alone: deferred updates only
  if (st->packed != 0 && st->packed != 1) return GFO_EINVAL;
  if (st->packed && st->delay == 0) return GFO_EINVAL;
  if (st->ldG < min_ld(p) || st->ldG % 64 != 0) return GFO_EINVAL;
  if (((uintptr_t)st->G & 15) != 0) return GFO_EINVAL;
  return GFO_OK;
}

static int validate_state(const gfo_problem* p, const gfo_state* st, Layout* L) {
  int rc = validate_state_fields(p, st);
  if (rc) return rc;
  if (!st->work || ((uintptr_t)st->work & 255) != 0) return GFO_EINVAL;
  *L = make_layout(p, st->ldG, st->kmax);
  if (st->work_bytes < L->total) return GFO_ENOSPC;
  return GFO_OK;
}

// validate_state for other sources of the library
int validate_job(const gfo_problem* p, const gfo_state* st, Layout* L) {
  int rc = validate_problem(p);
  if (rc) return rc;
  return validate_state(p, st, L);
}

static thread_local hipError_t t_last_hip = hipSuccess;

hipError_t note_hip(hipError_t e) {
  if (e != hipSuccess) t_last_hip = e;
  return e;
}

// The runtime keeps a failed call's error until it is read; one left by a call
// made before the entry point (by the caller or another library) is dropped
// here, so that the checks after this call's own launches report only them.
void discard_stale_hip() { (void)hipGetLastError(); }

}  // namespace gfo

using namespace gfo;

extern "C" {

const char* gfo_version(void) { return "libgfo 0.1 gfx950"; }

int32_t gfo_last_hip_error(const char** h_name) {
  const hipError_t e = t_last_hip;
  t_last_hip = hipSuccess;
  if (h_name) *h_name = hipGetErrorName(e);
  return (int32_t)e;
}

const char* gfo_strerror(int code) {
  switch (code) {
    case GFO_OK: return "ok";
    case GFO_EINVAL: return "invalid argument (sizes, null pointers or alignment)";
    case GFO_EHIP: return "a HIP runtime call or kernel launch failed";
    case GFO_ENOSPC: return "workspace too small";
    case GFO_ERANGE: return "more flipped pixels than the refresh workspace holds (kmax)";
    case GFO_ESCRATCH: return "problem too large for the library's static scratch";
    default: return "unknown error";
  }
}

// ldG argument of the size queries: 0 = the minimum, else checked like state.ldG
static int64_t query_ld(const gfo_problem* p, int64_t ldG) {
  if (ldG == 0) return min_ld(p);
  return ldG >= min_ld(p) && ldG % 64 == 0 ? ldG : -1;
}

int gfo_workspace_size(const gfo_problem* prob, int64_t ldG, int32_t kmax, size_t* h_bytes) {
  int rc = validate_problem(prob);
  if (rc) return rc;
  const int64_t ld = query_ld(prob, ldG);
  if (!h_bytes || kmax < 0 || ld < 0) return GFO_EINVAL;
  *h_bytes = make_layout(prob, ld, kmax).total;
  return GFO_OK;
}

int gfo_scores_offset(const gfo_problem* prob, int64_t ldG, int32_t kmax, size_t* h_offset) {
  int rc = validate_problem(prob);
  if (rc) return rc;
  const int64_t ld = query_ld(prob, ldG);
  if (!h_offset || kmax < 0 || ld < 0) return GFO_EINVAL;
  *h_offset = make_layout(prob, ld, kmax).scores;
  return GFO_OK;
}

int64_t gfo_min_ld(const gfo_problem* prob) {
  if (validate_problem(prob)) return -1;
  return min_ld(prob);
}

int gfo_g_elems(const gfo_problem* prob, int64_t ldG, int32_t packed, int64_t* h_elems) {
  int rc = validate_problem(prob);
  if (rc) return rc;
  const int64_t ld = query_ld(prob, ldG);
  if (!h_elems || ld < 0 || (packed != 0 && packed != 1)) return GFO_EINVAL;
  *h_elems = g_elems(packed, (int64_t)prob->ny * prob->nx, prob->n_mon, ld);
  return GFO_OK;
}

int init_G0(const gfo_problem* prob, gfo_state* st, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  const Geo g = make_geo(prob, st);
  char* w = (char*)st->work;
  // monitor coordinates travel with the call; wait for the copy so that the
  // caller's host array need not outlive it
  if (note_hip(hipMemcpyAsync(w + L.mon_xy, prob->h_mon_xy, (size_t)prob->n_mon * 2 * sizeof(double),
                              hipMemcpyHostToDevice, stream)) != hipSuccess)
    return GFO_EHIP;
  if (launch_init(g, st, L, stream) != hipSuccess) return GFO_EHIP;
  if (launch_dl_reset(g, st, L, stream) != hipSuccess) return GFO_EHIP;
  st->pending_calls = 0;
  // deferred mode, or a caller that asked for it (lower_stale = 1 on entry),
  // keeps the upper triangle of the design block alone
  st->lower_stale = g.upper;
  if (note_hip(hipStreamSynchronize(stream)) != hipSuccess) return GFO_EHIP;
  return GFO_OK;
}

int score_candidates(const gfo_problem* prob, const gfo_state* st, uint32_t cand_mask, double tau,
                     int32_t topk, int32_t min_spacing, gfo_pick* d_out, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  if (!d_out || topk < 1 || topk > GFO_MAX_RANK_K || min_spacing < 0 || !(tau >= 0.0) ||
      !(tau < 1.0))
    return GFO_EINVAL;
  if ((cand_mask & ((1u << prob->n_eps) - 1u)) == 0) return GFO_EINVAL;
  const Geo g = make_geo(prob, st);
  if (launch_score(g, st, L, cand_mask & ((1u << prob->n_eps) - 1u), tau, topk, min_spacing, d_out,
                   stream) != hipSuccess)
    return GFO_EHIP;
  return GFO_OK;
}

int apply_flip(const gfo_problem* prob, gfo_state* st, const gfo_pick* d_pick, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  if (!d_pick) return GFO_EINVAL;
  const Geo g = make_geo(prob, st);
  if (launch_apply(g, st, L, d_pick, stream) != hipSuccess) return GFO_EHIP;
  if (st->delay > 0 && ++st->pending_calls >= st->delay) {
    if (launch_flush(g, st, L, stream) != hipSuccess) return GFO_EHIP;
    st->pending_calls = 0;
  }
  return GFO_OK;
}

int gfo_flush(const gfo_problem* prob, gfo_state* st, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  if (st->delay == 0 || st->pending_calls == 0) return GFO_OK;
  const Geo g = make_geo(prob, st);
  if (launch_flush(g, st, L, stream) != hipSuccess) return GFO_EHIP;
  st->pending_calls = 0;
  return GFO_OK;
}

int gfo_sync_lower(const gfo_problem* prob, gfo_state* st, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  if (st->packed) return GFO_EINVAL;   // no lower triangle is stored
  if (!st->lower_stale) return GFO_OK;
  const Geo g = make_geo(prob, st);
  if (launch_sync_lower(g, st, stream) != hipSuccess) return GFO_EHIP;
  st->lower_stale = 0;
  return GFO_OK;
}

int gfo_greedy_steps(const gfo_problem* prob, gfo_state* st, int32_t n_steps, uint32_t cand_mask,
                     double tau, gfo_pick* d_picks, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  if (n_steps < 0 || !(tau >= 0.0) || !(tau < 1.0)) return GFO_EINVAL;
  const uint32_t mask = cand_mask & ((1u << prob->n_eps) - 1u);
  if (mask == 0) return GFO_EINVAL;
  if (n_steps == 0) return GFO_OK;
  const Geo g = make_geo(prob, st);
  gfo_pick* internal = (gfo_pick*)((char*)st->work + L.picks);
  if (st->delay > 0 && g_loop_form.load() == 0 && one_kernel_loop(g)) {
    // one kernel per move (pick, gather, elementwise part, next scores)
    const bool c64 = g.dtype == GFO_C64;
    if ((c64 ? launch_move_scores<float2>(g, st, L, mask, tau, stream)
             : launch_move_scores<double2>(g, st, L, mask, tau, stream)) != hipSuccess)
      return GFO_EHIP;
    for (int t = 0; t < n_steps; ++t) {
      int flushed = 0;
      if (st->pending_calls >= st->delay) {
        // the previous move's pivot values and the term count reach memory
        // before the flush
        if (t > 0 && (c64 ? launch_move_finish<float2>(g, st, L, t - 1, stream)
                          : launch_move_finish<double2>(g, st, L, t - 1, stream)) != hipSuccess)
          return GFO_EHIP;
        if (launch_flush(g, st, L, stream) != hipSuccess) return GFO_EHIP;
        st->pending_calls = 0;
        flushed = 1;
      }
      gfo_pick* pk = d_picks ? d_picks + t : internal;
      if ((c64 ? launch_move<float2>(g, st, L, t, flushed, mask, tau, pk, stream)
               : launch_move<double2>(g, st, L, t, flushed, mask, tau, pk, stream)) != hipSuccess)
        return GFO_EHIP;
      ++st->pending_calls;
    }
    if ((c64 ? launch_move_finish<float2>(g, st, L, n_steps - 1, stream)
             : launch_move_finish<double2>(g, st, L, n_steps - 1, stream)) != hipSuccess)
      return GFO_EHIP;
    if (st->pending_calls >= st->delay) {
      if (launch_flush(g, st, L, stream) != hipSuccess) return GFO_EHIP;
      st->pending_calls = 0;
    }
    return GFO_OK;
  }
  const bool fused = st->delay > 0 && (g.N + kScoreThreads - 1) / kScoreThreads <= kScoreMaxBlocks;
  if (!fused) {
    for (int t = 0; t < n_steps; ++t) {
      gfo_pick* pk = d_picks ? d_picks + t : internal;
      if (launch_score(g, st, L, mask, tau, 1, 0, pk, stream) != hipSuccess) return GFO_EHIP;
      if (launch_apply(g, st, L, pk, stream) != hipSuccess) return GFO_EHIP;
      if (st->delay > 0 && ++st->pending_calls >= st->delay) {
        if (launch_flush(g, st, L, stream) != hipSuccess) return GFO_EHIP;
        st->pending_calls = 0;
      }
    }
    return GFO_OK;
  }
  for (int t = 0; t < n_steps; ++t) {
    // a full term buffer is flushed after the previous move's elementwise part
    // (which sets the term count) and before this move's gather
    const bool flush = st->pending_calls >= st->delay;
    gfo_pick* pk = d_picks ? d_picks + t : internal;
    const hipError_t e =
        g.dtype == GFO_C64
            ? launch_fused_move<float2>(g, st, L, t > 0, mask, tau, pk, flush, stream)
            : launch_fused_move<double2>(g, st, L, t > 0, mask, tau, pk, flush, stream);
    if (e != hipSuccess) return GFO_EHIP;
    if (flush) st->pending_calls = 0;
    ++st->pending_calls;
  }
  const hipError_t e = g.dtype == GFO_C64 ? launch_fused_finish<float2>(g, st, L, stream)
                                          : launch_fused_finish<double2>(g, st, L, stream);
  if (e != hipSuccess) return GFO_EHIP;
  if (st->pending_calls >= st->delay) {
    if (launch_flush(g, st, L, stream) != hipSuccess) return GFO_EHIP;
    st->pending_calls = 0;
  }
  return GFO_OK;
}

static int validate_regions(const gfo_problem* prob, int32_t region) {
  if (region != region_side() || prob->ny % region || prob->nx % region) return GFO_EINVAL;
  const int64_t n = (int64_t)(prob->ny / region) * (prob->nx / region);
  if ((n + kScoreThreads - 1) / kScoreThreads > kScoreMaxBlocks) return GFO_EINVAL;
  return GFO_OK;
}

int score_regions(const gfo_problem* prob, const gfo_state* st, int32_t region,
                  uint32_t cand_mask, double tau, gfo_pick* d_out, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  if ((rc = validate_regions(prob, region))) return rc;
  if (!d_out || !(tau >= 0.0) || !(tau < 1.0)) return GFO_EINVAL;
  const uint32_t mask = cand_mask & ((1u << prob->n_eps) - 1u);
  if (mask == 0) return GFO_EINVAL;
  const Geo g = make_geo(prob, st);
  if (launch_score_regions(g, st, L, mask, tau, d_out, stream) != hipSuccess) return GFO_EHIP;
  return GFO_OK;
}

int gfo_region_pixels(const gfo_problem* prob, const gfo_state* st, int32_t region,
                      const gfo_pick* d_region, gfo_pick* d_pixels, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  if ((rc = validate_regions(prob, region))) return rc;
  if (!d_region || !d_pixels) return GFO_EINVAL;
  const Geo g = make_geo(prob, st);
  if (launch_region_pixels(g, st, d_region, d_pixels, stream) != hipSuccess) return GFO_EHIP;
  return GFO_OK;
}

int gfo_choose_eps_greedy(const gfo_pick* d_top, int32_t k, double eps, double u_explore,
                          double u_choice, gfo_pick* d_out, hipStream_t stream) {
  discard_stale_hip();
  if (!d_top || !d_out || k < 1 || k > GFO_MAX_RANK_K || !(eps >= 0.0 && eps <= 1.0) ||
      !(u_explore >= 0.0 && u_explore < 1.0) || !(u_choice >= 0.0 && u_choice < 1.0))
    return GFO_EINVAL;
  if (launch_choose_eps_greedy(d_top, k, eps, u_explore, u_choice, d_out, stream) != hipSuccess)
    return GFO_EHIP;
  return GFO_OK;
}

int apply_flips_rank_k(const gfo_problem* prob, gfo_state* st, const gfo_pick* d_picks, int32_t k,
                       int32_t gemm_precision, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  if (!d_picks || k < 1 || k > GFO_MAX_RANK_K || prob->dtype != GFO_C64 ||
      (gemm_precision != GFO_FP32 && gemm_precision != GFO_BF16))
    return GFO_EINVAL;
  if (st->packed) return GFO_EINVAL;   // the rank-k update streams whole rows
  const Geo g = make_geo(prob, st);
  if (st->delay > 0 && st->pending_calls > 0) {
    if (launch_flush(g, st, L, stream) != hipSuccess) return GFO_EHIP;
    st->pending_calls = 0;
  }
  if (launch_rank_k(g, st, L, d_picks, k, gemm_precision, stream) != hipSuccess) return GFO_EHIP;
  return GFO_OK;
}

int refresh_G(const gfo_problem* prob, gfo_state* st, hipStream_t stream) {
  discard_stale_hip();
  int rc = validate_problem(prob);
  if (rc) return rc;
  Layout L;
  if ((rc = validate_state(prob, st, &L))) return rc;
  const Geo g = make_geo(prob, st);
  // the flipped set is counted first: a set larger than kmax is refused before
  // anything of the state changes (pending deferred terms included)
  int32_t k = 0;
  if ((rc = launch_refresh_count(g, st, L, stream, &k))) return rc;
  if (k > st->kmax) {
    if (launch_refresh_overflow(st, stream) != hipSuccess) return GFO_EHIP;
    return GFO_ERANGE;
  }
  if (launch_dl_reset(g, st, L, stream) != hipSuccess) return GFO_EHIP;   // pending terms discarded
  st->pending_calls = 0;
  rc = launch_refresh(g, st, L, k, stream);
  // every entry rebuilt, or (deferred mode, or lower_stale = 1 on entry) the
  // upper triangle of the design block
  if (rc == GFO_OK) st->lower_stale = g.upper;
  return rc;
}

// Autotuner hooks: variants of the streaming rank-1 kernel.
int gfo_k1_variant_count(int32_t dtype) { return k1_variant_count(dtype); }
const char* gfo_k1_variant_name(int32_t dtype, int32_t idx) { return k1_variant_name(dtype, idx); }
int gfo_k1_set_variant(int32_t dtype, int32_t idx) { return k1_set_variant(dtype, idx); }
int gfo_k1_get_variant(int32_t dtype) { return k1_get_variant(dtype); }

int gfo_rk_variant_count(void) { return rk_variant_count(); }
const char* gfo_rk_variant_name(int32_t idx) { return rk_variant_name(idx); }
int gfo_rk_set_variant(int32_t idx) { return rk_set_variant(idx); }
int gfo_rk_get_variant(void) { return rk_get_variant(); }

int gfo_flush_variant_count(void) { return flush_variant_count(); }
const char* gfo_flush_variant_name(int32_t idx) { return flush_variant_name(idx); }
int gfo_flush_set_variant(int32_t idx) { return flush_set_variant(idx); }
int gfo_flush_get_variant(void) { return flush_get_variant(); }

int gfo_loop_set_form(int32_t form) {
  if (form != 0 && form != 1) return GFO_EINVAL;
  g_loop_form.store(form);
  return GFO_OK;
}
int gfo_loop_get_form(void) { return g_loop_form.load(); }

int gfo_time_next_k1(hipEvent_t before, hipEvent_t after) {
  if ((before == nullptr) != (after == nullptr)) return GFO_EINVAL;
  k1_time_next(before, after);
  return GFO_OK;
}

}  // extern "C"
