// One greedy step: candidate scores + selection, move snapshot, pivot gather
// and the streaming rank-1 Dyson update of G.
//
// Scores follow paper eqs. form4-form9 for a one-pixel region evaluated at the
// FOM monitor (eq. para1); the update is eq. form10 with the one-pixel solve of
// eq. form14, i.e. G += c G[:, j] G[j, :] with c = alpha / (1 - alpha G_jj).
#include "gfo_internal.hpp"

#include <atomic>
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
  const T* __restrict__ grow = G + (int64_t)(g.N + g.m0) * g.ld;
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
  return hipGetLastError();
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

// ------------------------------------------------------------------ K1: rank-1 update
// G[r, q] += cu[r] * v[q] over all R rows and ld columns (v is zero beyond N).
// Workgroup tile: RB rows x (256 threads x 16 bytes).  Each thread keeps its
// 16-byte slice of v in registers and streams RB rows of G through it, U rows
// in flight at a time; cu[r] is uniform across the workgroup.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float2> {
  using type = f32x4;
  static constexpr int n = 2;
  __device__ __forceinline__ static f32x4 fma(float2 c, f32x4 v, f32x4 g) {
    g.x = fmaf(c.x, v.x, g.x); g.x = fmaf(-c.y, v.y, g.x);
    g.y = fmaf(c.x, v.y, g.y); g.y = fmaf(c.y, v.x, g.y);
    g.z = fmaf(c.x, v.z, g.z); g.z = fmaf(-c.y, v.w, g.z);
    g.w = fmaf(c.x, v.w, g.w); g.w = fmaf(c.y, v.z, g.w);
    return g;
  }
};
template <> struct Vec16<double2> {
  using type = f64x2;
  static constexpr int n = 1;
  __device__ __forceinline__ static f64x2 fma(double2 c, f64x2 v, f64x2 g) {
    g.x = fma_d(c.x, v.x, g.x); g.x = fma_d(-c.y, v.y, g.x);
    g.y = fma_d(c.x, v.y, g.y); g.y = fma_d(c.y, v.x, g.y);
    return g;
  }
  __device__ __forceinline__ static double fma_d(double a, double b, double c) { return ::fma(a, b, c); }
};

constexpr int kK1Threads = 256;

// Workgroup tile: RB rows x (256 threads x CPT chunks x 16 bytes).  Thread t
// owns chunks at column offsets (t + c*256)*VN, c < CPT, so every load
// instruction of the workgroup covers 4 KB of one row contiguously.  U rows
// are in flight per batch; PIPE = true issues the loads of the next batch
// before the stores of the current one.
template <typename T, int RB, int U, int CPT, bool NT, bool PIPE>
__device__ __forceinline__ void k_rank1_tile(int R, int64_t ld, int ct, int64_t rt,
                                             const T* __restrict__ cu, const T* __restrict__ v,
                                             T* __restrict__ G);

// Tiles are visited grid-stride (tile = blockIdx.x, blockIdx.x + gridDim.x, ...), so
// the launch can stay below the 2^32 work-item limit of one dispatch on any shape.
template <typename T, int RB, int U, int CPT, bool NT, bool PIPE>
__global__ __launch_bounds__(kK1Threads) void k_rank1(int R, int64_t ld, int ncoltiles,
                                                      int64_t ntiles,
                                                      const Snap* __restrict__ snap,
                                                      const T* __restrict__ cu,
                                                      const T* __restrict__ v, T* __restrict__ G) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  static_assert(RB % U == 0, "RB must be a multiple of U");
  if (snap->j < 0) return;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    k_rank1_tile<T, RB, U, CPT, NT, PIPE>(R, ld, (int)(tile % ncoltiles), tile / ncoltiles, cu, v, G);
  }
}

template <typename T, int RB, int U, int CPT, bool NT, bool PIPE>
__device__ __forceinline__ void k_rank1_tile(int R, int64_t ld, int ct, int64_t rt,
                                             const T* __restrict__ cu, const T* __restrict__ v,
                                             T* __restrict__ G) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  const int64_t qb = (int64_t)ct * (kK1Threads * VN * CPT) + threadIdx.x * VN;
  V vv[CPT];
  bool ok[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int64_t q = qb + (int64_t)c * kK1Threads * VN;
    ok[c] = q < ld;
    vv[c] = ok[c] ? *reinterpret_cast<const V*>(v + q) : V{};
  }
  const int r0 = (int)(rt * RB);
  auto load_batch = [&](int rr, V (&gv)[U][CPT], T (&cv)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + rr + u;
      if (r < R) {
        cv[u] = cu[r];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          if (ok[c]) {
            V* p = reinterpret_cast<V*>(G + (int64_t)r * ld + qb + (int64_t)c * kK1Threads * VN);
            gv[u][c] = NT ? __builtin_nontemporal_load(p) : *p;
          }
        }
      }
    }
  };
  auto store_batch = [&](int rr, V (&gv)[U][CPT], T (&cv)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + rr + u;
      if (r < R) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          if (ok[c]) {
            V* p = reinterpret_cast<V*>(G + (int64_t)r * ld + qb + (int64_t)c * kK1Threads * VN);
            const V o = Vec16<T>::fma(cv[u], vv[c], gv[u][c]);
            if (NT) __builtin_nontemporal_store(o, p); else *p = o;
          }
        }
      }
    }
  };
  if constexpr (!PIPE) {
#pragma unroll 1
    for (int rr = 0; rr < RB; rr += U) {
      V gv[U][CPT];
      T cv[U];
      load_batch(rr, gv, cv);
      store_batch(rr, gv, cv);
    }
  } else {
    V ga[U][CPT], gb[U][CPT];
    T ca[U], cb[U];
    load_batch(0, ga, ca);
#pragma unroll 1
    for (int rr = 0; rr < RB; rr += 2 * U) {
      if (rr + U < RB) load_batch(rr + U, gb, cb);
      store_batch(rr, ga, ca);
      if (rr + U < RB) {
        if (rr + 2 * U < RB) load_batch(rr + 2 * U, ga, ca);
        store_batch(rr + U, gb, cb);
      }
    }
  }
}

struct K1Variant {
  const char* name;
  void (*launch)(int R, int64_t ld, const Snap*, const void*, const void*, void*, hipStream_t);
};

// at most MAXB workgroups per launch (4M x 256 work-items stays far below 2^32)
template <typename T, int RB, int U, int CPT, bool NT, bool PIPE, int64_t MAXB = (int64_t)1 << 22>
static void launch_k1(int R, int64_t ld, const Snap* snap, const void* cu, const void* v, void* G,
                      hipStream_t s) {
  constexpr int VN = Vec16<T>::n;
  constexpr int cols = kK1Threads * VN * CPT;
  const int ncol = (int)((ld + cols - 1) / cols);
  const int64_t nrow = (R + RB - 1) / RB;
  const int64_t ntiles = (int64_t)ncol * nrow;
  const int64_t nblk = ntiles < MAXB ? ntiles : MAXB;
  hipLaunchKernelGGL((k_rank1<T, RB, U, CPT, NT, PIPE>), dim3((unsigned)nblk), dim3(kK1Threads), 0,
                     s, R, ld, ncol, ntiles, snap, (const T*)cu, (const T*)v, (T*)G);
}

// name: rows-per-workgroup x rows-in-flight x 16B-chunks-per-thread [_nt] [_pipe]
// [_gB: at most B workgroups, each walking many tiles].
// Entry 0 is the default: the fastest on the 128x128 and 48x2048 problems on
// MI355X for both storage types (2 rows per short-lived workgroup, non-temporal
// loads and stores).
#define K1V(T, RB, U, CPT, NT, PIPE, NAME) {NAME, launch_k1<T, RB, U, CPT, NT, PIPE>}
#define K1G(T, RB, U, CPT, NT, PIPE, MAXB, NAME) {NAME, launch_k1<T, RB, U, CPT, NT, PIPE, MAXB>}
#define K1_TABLE(T)                                                                         \
  {                                                                                         \
    K1V(T, 2, 2, 1, true, false, "2x2x1_nt"), K1V(T, 4, 4, 1, true, false, "4x4x1_nt"),     \
    K1V(T, 1, 1, 1, true, false, "1x1x1_nt"), K1V(T, 2, 2, 2, true, false, "2x2x2_nt"),     \
    K1V(T, 1, 1, 2, true, false, "1x1x2_nt"), K1V(T, 2, 1, 1, true, false, "2x1x1_nt"),     \
    K1V(T, 16, 8, 1, false, false, "16x8x1"), K1V(T, 32, 8, 1, false, false, "32x8x1"),     \
    K1V(T, 16, 8, 1, true, false, "16x8x1_nt"), K1V(T, 32, 8, 1, true, false, "32x8x1_nt"), \
    K1V(T, 64, 16, 1, false, false, "64x16x1"), K1V(T, 8, 8, 1, false, false, "8x8x1"),     \
    K1V(T, 32, 16, 1, true, false, "32x16x1_nt"), K1V(T, 64, 8, 1, true, false, "64x8x1_nt"), \
    K1V(T, 16, 4, 2, false, false, "16x4x2"), K1V(T, 32, 4, 2, true, false, "32x4x2_nt"),   \
    K1V(T, 16, 8, 2, false, false, "16x8x2"), K1V(T, 64, 4, 4, false, false, "64x4x4"),     \
    K1V(T, 4, 4, 4, false, false, "4x4x4"), K1V(T, 2, 2, 8, false, false, "2x2x8"),         \
    K1V(T, 1, 1, 16, false, false, "1x1x16"), K1V(T, 32, 4, 1, false, true, "32x4x1_pipe"), \
    K1V(T, 64, 8, 1, false, true, "64x8x1_pipe"), K1V(T, 32, 4, 2, false, true, "32x4x2_pipe"), \
    K1V(T, 64, 8, 1, true, true, "64x8x1_nt_pipe"), K1V(T, 16, 2, 4, true, true, "16x2x4_nt_pipe"), \
    K1V(T, 8, 8, 1, true, false, "8x8x1_nt"),                                              \
    K1V(T, 8, 4, 2, true, false, "8x4x2_nt"), K1V(T, 4, 4, 2, true, false, "4x4x2_nt"),       \
    K1V(T, 8, 8, 2, true, false, "8x8x2_nt"), K1V(T, 2, 2, 4, true, false, "2x2x4_nt"),       \
    K1V(T, 16, 16, 1, true, false, "16x16x1_nt"), K1V(T, 4, 4, 4, true, false, "4x4x4_nt"),   \
    K1V(T, 32, 8, 1, true, true, "32x8x1_nt_pipe"), K1V(T, 16, 4, 1, true, true, "16x4x1_nt_pipe"), \
    K1G(T, 2, 1, 1, true, false, 64, "2x1x1_nt_g64"),                                      \
  }
static const K1Variant kK1c64[] = K1_TABLE(float2);
static const K1Variant kK1c128[] = K1_TABLE(double2);
#undef K1_TABLE
#undef K1G
#undef K1V
static std::atomic<int> g_k1_sel[2] = {{0}, {0}};
static std::atomic<hipEvent_t> g_k1_before{nullptr}, g_k1_after{nullptr};

void k1_time_next(hipEvent_t before, hipEvent_t after) {
  g_k1_after.store(after);
  g_k1_before.store(before);
}

void k1_take_timing(hipEvent_t* before, hipEvent_t* after) {
  *before = g_k1_before.exchange(nullptr);
  *after = g_k1_after.exchange(nullptr);
}

static const K1Variant* k1_table(int dtype, int* n) {
  if (dtype == GFO_C64) {
    *n = (int)(sizeof(kK1c64) / sizeof(kK1c64[0]));
    return kK1c64;
  }
  *n = (int)(sizeof(kK1c128) / sizeof(kK1c128[0]));
  return kK1c128;
}
int k1_variant_count(int dtype) {
  int n;
  k1_table(dtype, &n);
  return n;
}
const char* k1_variant_name(int dtype, int idx) {
  int n;
  const K1Variant* t = k1_table(dtype, &n);
  return (idx >= 0 && idx < n) ? t[idx].name : nullptr;
}
int k1_set_variant(int dtype, int idx) {
  int n;
  k1_table(dtype, &n);
  if (idx < 0 || idx >= n || (dtype != GFO_C64 && dtype != GFO_C128)) return GFO_EINVAL;
  g_k1_sel[dtype].store(idx);
  return GFO_OK;
}
int k1_get_variant(int dtype) { return g_k1_sel[dtype == GFO_C64 ? 0 : 1].load(); }

// ------------------------------------------------------------------ launchers
template <typename T>
static hipError_t score_typed(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                              double tau, int topk, int spacing, gfo_pick* out, hipStream_t s) {
  char* w = (char*)st->work;
  int nblk = (g.N + kScoreThreads - 1) / kScoreThreads;
  if (nblk > kScoreMaxBlocks) nblk = kScoreMaxBlocks;
  hipLaunchKernelGGL(k_score<T>, dim3(nblk), dim3(kScoreThreads), 0, s, g, (const T*)st->G,
                     (const T*)st->E, (const double2*)st->diag64, (const uint8_t*)st->eps_idx, mask,
                     tau, (double*)(w + L.scores), (double*)(w + L.partial), (int*)(w + L.pfirst),
                     st->status);
  // the greedy pick reads the workgroup summaries (one wave); the spaced top-k
  // rescans every score after each pick
  const int sel_threads = topk == 1 ? 64 : kSelectThreads;
  hipLaunchKernelGGL(k_select<T>, dim3(1), dim3(sel_threads), 0, s, g, (const T*)st->E,
                     (double*)(w + L.scores), (const double*)(w + L.partial),
                     (const int*)(w + L.pfirst), nblk, tau, topk, spacing, out);
  return hipGetLastError();
}

hipError_t launch_score(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                        double tau, int topk, int spacing, gfo_pick* out, hipStream_t s) {
  if (g.dtype == GFO_C64) return score_typed<float2>(g, st, L, mask, tau, topk, spacing, out, s);
  return score_typed<double2>(g, st, L, mask, tau, topk, spacing, out, s);
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
  int nv;
  const K1Variant* tab = k1_table(g.dtype, &nv);
  hipEvent_t before, after;
  k1_take_timing(&before, &after);
  if (before && hipEventRecord(before, s) != hipSuccess) return hipErrorUnknown;
  tab[k1_get_variant(g.dtype)].launch(g.R, g.ld, snap, cu, v, st->G, s);
  if (after && hipEventRecord(after, s) != hipSuccess) return hipErrorUnknown;
  return hipGetLastError();
}

hipError_t launch_apply(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                        hipStream_t s) {
  if (g.dtype == GFO_C64) return apply_typed<float2>(g, st, L, pick, s);
  return apply_typed<double2>(g, st, L, pick, s);
}

}  // namespace gfo
