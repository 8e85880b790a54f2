// One greedy step: candidate scores + selection, move snapshot and pivot gather;
// the streaming rank-1 Dyson update of G itself is in gfo_rank1.hip.
//
// Scores follow paper eqs. form4-form9 for a one-pixel region evaluated at the
// FOM monitor (eq. para1); the update is eq. form10 with the one-pixel solve of
// eq. form14, i.e. G += c G[:, j] G[j, :] with c = alpha / (1 - alpha G_jj).
#include "gfo_internal.hpp"

#include <math.h>

namespace gfo {

// ------------------------------------------------------------------ K3: scores
// One thread per pixel (grid-stride).  Writes every (pixel, material) score,
// -inf for non-candidates, and per workgroup its best score and, when every
// thread scored one pixel, the lowest index within the tie band of that best.
template <typename T>
__global__ __launch_bounds__(kScoreThreads) void k_score(
    Geo g, const T* __restrict__ G, const T* __restrict__ E, const double2* __restrict__ diag64,
    const uint8_t* __restrict__ eps_idx, uint32_t mask, double tau, double* __restrict__ scores,
    double* __restrict__ partial, int* __restrict__ pfirst, int32_t* __restrict__ status) {
  __shared__ double sh[kScoreThreads / 64];
  __shared__ int shi[kScoreThreads / 64];
  const double2 Em0 = St<T>::to_d(E[g.N + g.m0]);
  const T* __restrict__ grow = G + g_off(g, g.N + g.m0, 0);
  double best = -INFINITY;
  bool bad = false;
  double F[GFO_MAX_EPS];
  const int p0 = blockIdx.x * blockDim.x + threadIdx.x;
  for (int p = p0; p < g.N; p += gridDim.x * blockDim.x) {
    const int cur = eps_idx[p];
    const double2 d = diag64[p];
    const double2 gE = cmul(St<T>::to_d(grow[p]), St<T>::to_d(E[p]));
    best = fmax(best, score_pixel(g, p, cur, d, gE, Em0, mask, scores, &bad, F));
  }
  const bool one_pixel_each = (int64_t)gridDim.x * blockDim.x >= g.N;
  score_block_end(g, best, p0, one_pixel_each, F, tau, partial, pfirst, gridDim.x, sh, shi);
  if (bad) atomicOr(status, GFO_STATUS_NONFINITE);
}

// ------------------------------------------------------------------ K3b: selection
// Single workgroup.  Greedy rule with the relative tie band tau and the
// lowest-(pixel, material) winner, repeated topk times with the spacing
// exclusion.  Modifies `scores` (marks excluded candidates -inf).
template <typename T>
__global__ __launch_bounds__(kSelectThreads) void k_select(
    Geo g, const T* __restrict__ E, double* __restrict__ scores, const double* __restrict__ partial,
    const int* __restrict__ pfirst, int nblk, double tau, int topk, int spacing,
    gfo_pick* __restrict__ out) {
  __shared__ double shd[kSelectThreads / 64];
  __shared__ int shi[kSelectThreads / 64];
  const double fom = cabs2(St<T>::to_d(E[g.N + g.m0]));
  if (topk == 1 && nblk * kScoreThreads >= g.N) {
    // the greedy pick of the fused loop (one pixel per score thread)
    const gfo_pick pk = greedy_pick_block(g, fom, scores, partial, pfirst, nblk, tau, shd, shi);
    if (threadIdx.x == 0) out[0] = pk;
    return;
  }
  const int total = g.N * g.n_eps;
  const int win = spacing > 1 ? spacing - 1 : 0;
  int t = 0;
  if (nblk * kScoreThreads >= g.N && blockDim.x == kSelectThreads) {
    // One pixel per score thread: workgroup b's scores are [b span, b span + span),
    // partial[b] their maximum and pfirst[b] the lowest index within the tie band
    // of that maximum.  Both summaries stay in LDS.  A pick takes the first chunk
    // whose maximum reaches the band; if that chunk holds the global maximum its
    // summary is the winner (the same decision as greedy_pick_block), otherwise
    // (a near-tie across chunks) the chunk is scanned.  After the exclusion the
    // chunks it touched are summarised again, two at a time, 512 threads and at
    // most kSelVals scores per thread each.
    static_assert(kSelectThreads == 1024, "two groups of eight waves");
    constexpr int kSelVals = kScoreThreads * GFO_MAX_EPS / 512;
    __shared__ double spart[kScoreMaxBlocks];
    __shared__ int sfirst[kScoreMaxBlocks];
    __shared__ double gm[kSelectThreads / 64];
    __shared__ int gf[kSelectThreads / 64];
    const int span = kScoreThreads * g.n_eps;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
      spart[i] = partial[i];
      sfirst[i] = pfirst[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = threadIdx.x >> 9, gi = threadIdx.x & 511;   // two groups of eight waves
    for (; t < topk; ++t) {
      double m = -INFINITY;
      for (int i = threadIdx.x; i < nblk; i += blockDim.x) m = fmax(m, spart[i]);
      m = block_max(m, shd);
      if (!(m > fom * (1.0 + tau))) break;
      const double thr = tie_threshold(m, tau);
      int bq = 0x7fffffff;
      for (int i = threadIdx.x; i < nblk; i += blockDim.x)
        if (spart[i] >= thr) {
          bq = i;
          break;
        }
      bq = block_min(bq, shi);
      if (bq == 0x7fffffff) break;                    // non-finite scores
      int first = sfirst[bq];
      if (!(spart[bq] == m) || first == 0x7fffffff) {
        const int lo = bq * span, hi = min(lo + span, total);
        int f = 0x7fffffff;
        for (int i = lo + threadIdx.x; i < hi; i += blockDim.x)
          if (scores[i] >= thr) {
            f = i;
            break;
          }
        first = block_min(f, shi);
      }
      if (first == 0x7fffffff) break;
      const int j = first / g.n_eps;
      if (threadIdx.x == 0) {
        gfo_pick pk;
        pk.pixel = j;
        pk.eps_idx = first - j * g.n_eps;
        pk.fom_new = scores[first];
        pk.dfom = pk.fom_new - fom;
        out[t] = pk;
      }
      if (t + 1 < topk) {   // exclude the pick's window, then summarise the chunks it touched
        const int iy = j / g.nx, ix = j - (j / g.nx) * g.nx;
        const int w = 2 * win + 1;
        __syncthreads();
        for (int k = threadIdx.x; k < w * w * g.n_eps; k += blockDim.x) {
          const int e = k % g.n_eps, cell = k / g.n_eps;
          const int yy = iy - win + cell / w, xx = ix - win + cell % w;
          if (yy >= 0 && yy < g.ny && xx >= 0 && xx < g.nx)
            scores[(int64_t)(yy * g.nx + xx) * g.n_eps + e] = -INFINITY;
        }
        __syncthreads();
        const int b_lo = (max(iy - win, 0) * g.nx + max(ix - win, 0)) / kScoreThreads;
        const int b_hi = min((min(iy + win, g.ny - 1) * g.nx + min(ix + win, g.nx - 1)) / kScoreThreads, nblk - 1);
        for (int b0 = b_lo; b0 <= b_hi; b0 += 2) {       // uniform
          const int b = b0 + grp;
          const bool live = b <= b_hi;
          const int lo = b * span, hi = live ? min(lo + span, total) : lo;
          double v[kSelVals];
          double mb = -INFINITY;
#pragma unroll
          for (int q = 0; q < kSelVals; ++q) {
            const int i = lo + gi + 512 * q;
            v[q] = i < hi ? scores[i] : -INFINITY;
            mb = fmax(mb, v[q]);
          }
          mb = wave_max(mb);
          if (lane == 0) gm[wv] = mb;
          __syncthreads();
          mb = -INFINITY;
#pragma unroll
          for (int q = 0; q < 8; ++q) mb = fmax(mb, gm[8 * grp + q]);
          const double tb = tie_threshold(mb, tau);
          int fb = 0x7fffffff;
#pragma unroll
          for (int q = kSelVals - 1; q >= 0; --q)
            if (mb > -INFINITY && v[q] >= tb) fb = lo + gi + 512 * q;
          fb = wave_min(fb);
          if (lane == 0) gf[wv] = fb;
          __syncthreads();
          if (live && gi == 0) {
            int f = 0x7fffffff;
#pragma unroll
            for (int q = 0; q < 8; ++q) f = min(f, gf[8 * grp + q]);
            spart[b] = mb;
            sfirst[b] = f;
          }
        }
        __syncthreads();
      }
    }
  } else {
    for (; t < topk; ++t) {
      double m = -INFINITY;
      if (t == 0) {
        for (int i = threadIdx.x; i < nblk; i += blockDim.x) m = fmax(m, partial[i]);
      } else {
        for (int i = threadIdx.x; i < total; i += blockDim.x) m = fmax(m, scores[i]);
      }
      m = block_max(m, shd);
      if (!(m > fom * (1.0 + tau))) break;
      const double thr = m - tau * m;
      int first = 0x7fffffff;
      if (t == 0 && nblk * kScoreThreads >= g.N) {
        // score workgroup b covered pixels [b*256, b*256 + 256): only workgroups whose
        // maximum reaches the tie threshold can hold the winner; visit them in order
        const int span = kScoreThreads * g.n_eps;
        for (int b = 0; b < nblk; ++b) {
          if (!(partial[b] >= thr)) continue;          // uniform across the workgroup
          const int lo = b * span, hi = min(lo + span, total);
          int f = 0x7fffffff;
          for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            if (scores[i] >= thr) {
              f = i;
              break;
            }
          }
          f = block_min(f, shi);
          if (f != 0x7fffffff) {
            first = f;
            break;
          }
        }
      } else {
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
          if (scores[i] >= thr) {
            first = i;
            break;
          }
        }
        first = block_min(first, shi);
      }
      const int j = first / g.n_eps;
      if (threadIdx.x == 0) {
        gfo_pick pk;
        pk.pixel = j;
        pk.eps_idx = first - j * g.n_eps;
        pk.fom_new = scores[first];
        pk.dfom = pk.fom_new - fom;
        out[t] = pk;
      }
      if (t + 1 < topk) {
        __syncthreads();
        const int iy = j / g.nx, ix = j - (j / g.nx) * g.nx;
        const int w = 2 * win + 1;
        for (int k = threadIdx.x; k < w * w * g.n_eps; k += blockDim.x) {
          const int e = k % g.n_eps, cell = k / g.n_eps;
          const int yy = iy - win + cell / w, xx = ix - win + cell % w;
          if (yy >= 0 && yy < g.ny && xx >= 0 && xx < g.nx)
            scores[(int64_t)(yy * g.nx + xx) * g.n_eps + e] = -INFINITY;
        }
        __syncthreads();
      }
    }
  }
  if (threadIdx.x == 0) {
    for (; t < topk; ++t) {
      gfo_pick pk;
      pk.pixel = -1;
      pk.eps_idx = -1;
      pk.fom_new = fom;
      pk.dfom = 0.0;
      out[t] = pk;
    }
  }
}

// ------------------------------------------------------------------ policy
// Epsilon-greedy choice (Sec. V) among the records of a top-k selection: the
// improving moves come first (the greedy one at index 0), sentinels after.
__global__ void k_choose_eps_greedy(const gfo_pick* __restrict__ top, int k, double eps,
                                    double u_explore, double u_choice, gfo_pick* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int n = 0;
  while (n < k && top[n].pixel >= 0) ++n;
  int i = 0;
  if (n > 0 && u_explore < eps) {
    i = (int)(u_choice * (double)n);
    if (i > n - 1) i = n - 1;
  }
  *out = top[i];
}

hipError_t launch_choose_eps_greedy(const gfo_pick* top, int k, double eps, double u_explore,
                                    double u_choice, gfo_pick* out, hipStream_t s) {
  hipLaunchKernelGGL(k_choose_eps_greedy, dim3(1), dim3(64), 0, s, top, k, eps, u_explore, u_choice,
                     out);
  return note_hip(hipGetLastError());
}

// ------------------------------------------------------------------ K2a: snapshot
// Single thread.  Validates the pick, computes c in FP64 from diag64 and
// records the scalars the later kernels need before anything is overwritten.
template <typename T>
__global__ void k_snap(Geo g, const gfo_pick* __restrict__ pick, const T* __restrict__ E,
                       const double2* __restrict__ diag64, uint8_t* __restrict__ eps_idx,
                       int32_t* __restrict__ flips, int flip_cap, int32_t* __restrict__ n_flips,
                       int32_t* __restrict__ status, Snap* __restrict__ snap,
                       int32_t* __restrict__ dl_count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Snap s = {};
  s.j = -1;
  const int j = pick->pixel, e = pick->eps_idx;
  if (j >= 0 && j < g.N && e >= 0 && e < g.n_eps && e != (int)eps_idx[j]) {
    const double a = g.k0sq * (g.eps[e] - g.eps[eps_idx[j]]);
    const double2 d = diag64[j];
    const double2 den = make_double2(1.0 - a * d.x, -a * d.y);
    if (cabs2(den) < 1e-24) {
      atomicOr(status, GFO_STATUS_SINGULAR);
    } else {
      s.j = j;
      s.e_new = e;
      s.alpha = a;
      s.c = rdiv(a, den);
      s.Ej = St<T>::to_d(E[j]);
      s.dj = d;
      if (dl_count != nullptr) {             // deferred mode: this move's pending-term index
        s.slot = *dl_count;
        *dl_count = s.slot + 1;
      }
      eps_idx[j] = (uint8_t)e;
      const int n = *n_flips;
      if (n < flip_cap) {
        flips[2 * n] = j;
        flips[2 * n + 1] = e;
      } else {
        atomicOr(status, GFO_STATUS_HISTORY_FULL);
      }
      *n_flips = n + 1;
    }
  }
  *snap = s;
}

// ------------------------------------------------------------------ K2b: pivot gather
// Thread i: u_i = G[i, j] (column, all R rows) and v_i = G[j, i] (row, N
// columns) are copied to scratch (cu = c u) before K1 overwrites them, and the
// O(R) / O(N) parts of the update are applied here:
//   E_i += c u_i E_j,   diag64_i += c u_i v_i  (FP64),   diag64_j = d_j / (1 - alpha d_j).
template <typename T>
__global__ void k_gather(Geo g, const Snap* __restrict__ snap, const T* __restrict__ G,
                         T* __restrict__ E, double2* __restrict__ diag64, T* __restrict__ cu,
                         T* __restrict__ v) {
  const int j = snap->j;
  if (j < 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double2 c = snap->c;
  double2 cu_d = make_double2(0.0, 0.0);
  if (i < g.R) {
    const double2 u = (i == j) ? snap->dj : St<T>::to_d(G[g_at(g, i, j)]);
    cu_d = cmul(c, u);
    cu[i] = St<T>::from_d(cu_d);
    E[i] = St<T>::from_d(cadd(St<T>::to_d(E[i]), cmul(cu_d, snap->Ej)));
  }
  if (i < g.ld) {
    if (i < g.N) {
      const T vi = G[g_at(g, j, i)];
      v[i] = vi;
      if (i == j) {
        const double2 d = snap->dj;
        diag64[j] = cmul(d, rdiv(1.0, make_double2(1.0 - snap->alpha * d.x, -snap->alpha * d.y)));
      } else {
        diag64[i] = cadd(diag64[i], cmul(cu_d, St<T>::to_d(vi)));
      }
    } else {
      v[i] = St<T>::from_d(make_double2(0.0, 0.0));
    }
  }
}

// ------------------------------------------------------------------ launchers
template <typename T>
static hipError_t score_typed(const Geo& g, const gfo_state* st, const ScoreBufs& b, uint32_t mask,
                              double tau, int topk, int spacing, gfo_pick* out, hipStream_t s) {
  const int nblk = score_blocks(g);
  hipLaunchKernelGGL(k_score<T>, dim3(nblk), dim3(kScoreThreads), 0, s, g, (const T*)st->G,
                     (const T*)st->E, (const double2*)st->diag64, (const uint8_t*)st->eps_idx, mask,
                     tau, b.scores, b.partial, b.pfirst, st->status);
  // the greedy pick reads the workgroup summaries (one wave); the spaced top-k
  // rescans every score after each pick
  const int sel_threads = topk == 1 ? 64 : kSelectThreads;
  hipLaunchKernelGGL(k_select<T>, dim3(1), dim3(sel_threads), 0, s, g, (const T*)st->E, b.scores,
                     (const double*)b.partial, (const int*)b.pfirst, nblk, tau, topk, spacing, out);
  return note_hip(hipGetLastError());
}

hipError_t launch_score_into(const Geo& g, const gfo_state* st, const ScoreBufs& b, uint32_t mask,
                             double tau, int topk, int spacing, gfo_pick* out, hipStream_t s) {
  if (g.dtype == GFO_C64) return score_typed<float2>(g, st, b, mask, tau, topk, spacing, out, s);
  return score_typed<double2>(g, st, b, mask, tau, topk, spacing, out, s);
}

hipError_t launch_score(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                        double tau, int topk, int spacing, gfo_pick* out, hipStream_t s) {
  char* w = (char*)st->work;
  const ScoreBufs b{(double*)(w + L.scores), (double*)(w + L.partial), (int*)(w + L.pfirst)};
  return launch_score_into(g, st, b, mask, tau, topk, spacing, out, s);
}

template <typename T>
static hipError_t apply_typed(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                              hipStream_t s) {
  char* w = (char*)st->work;
  Snap* snap = (Snap*)(w + L.snap);
  T* cu = (T*)(w + L.cu);
  T* v = (T*)(w + L.v);
  if (st->delay > 0) return launch_apply_deferred<T>(g, st, L, pick, s);
  hipLaunchKernelGGL(k_snap<T>, dim3(1), dim3(64), 0, s, g, pick, (const T*)st->E,
                     (const double2*)st->diag64, st->eps_idx, st->flips, st->flip_cap, st->n_flips,
                     st->status, snap, (int32_t*)nullptr);
  const int64_t n = g.R > g.ld ? (int64_t)g.R : g.ld;
  hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                     (const Snap*)snap, (const T*)st->G, (T*)st->E, (double2*)st->diag64, cu, v);
  return launch_rank1(g, snap, cu, v, st->G, s);
}

hipError_t launch_apply(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                        hipStream_t s) {
  if (g.dtype == GFO_C64) return apply_typed<float2>(g, st, L, pick, s);
  return apply_typed<double2>(g, st, L, pick, s);
}

}  // namespace gfo
