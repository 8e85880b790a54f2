// The streaming rank-1 Dyson update of G (eq. form10 with the one-pixel solve
// of eq. form14): G[r, q] += cu[r] v[q] over all rows and columns, with
// cu = c G[:, j] and v = G[j, :] gathered beforehand.  One pass over G in HBM;
// tile variants are selected by the autotuner.
#include "gfo_internal.hpp"

#include <atomic>

namespace gfo {

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
// upper: only the upper triangle of the design block is kept current (the
// block is symmetric; readers take (min, max)), so the tiles of design rows that
// lie wholly below its diagonal are left out of the enumeration (ntiles counts
// the others); monitor rows are always updated.
template <typename T, int RB, int U, int CPT, bool NT, bool PIPE>
__global__ __launch_bounds__(kK1Threads) void k_rank1(int R, int64_t ld, int ncoltiles,
                                                      int64_t ntiles, int N, int upper,
                                                      const Snap* __restrict__ snap,
                                                      const T* __restrict__ cu,
                                                      const T* __restrict__ v, T* __restrict__ G) {
  static_assert(RB % U == 0, "RB must be a multiple of U");
  constexpr int64_t cols = (int64_t)kK1Threads * Vec16<T>::n * CPT;
  if (snap->j < 0) return;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int rt, ct;
    ut_group(tile, ncoltiles, upper ? N / RB : 0, RB, (int)cols, rt, ct);
    k_rank1_tile<T, RB, U, CPT, NT, PIPE>(R, ld, ct, rt, cu, v, G);
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
  void (*launch)(int R, int64_t ld, int N, int upper, const Snap*, const void*, const void*, void*,
                 hipStream_t);
};

// at most MAXB workgroups per launch (4M x 256 work-items stays far below 2^32)
template <typename T, int RB, int U, int CPT, bool NT, bool PIPE, int64_t MAXB = (int64_t)1 << 22>
static void launch_k1(int R, int64_t ld, int N, int upper, const Snap* snap, const void* cu,
                      const void* v, void* G, hipStream_t s) {
  constexpr int VN = Vec16<T>::n;
  constexpr int cols = kK1Threads * VN * CPT;
  const int ncol = (int)((ld + cols - 1) / cols);
  const int64_t nrow = (R + RB - 1) / RB;
  static_assert(cols % RB == 0 || RB % cols == 0, "tile rows and columns must be powers of two");
  const int64_t ntiles = ut_group_count((int)nrow, ncol, upper ? N / RB : 0, RB, cols);
  const int64_t nblk = ntiles < MAXB ? ntiles : MAXB;
  hipLaunchKernelGGL((k_rank1<T, RB, U, CPT, NT, PIPE>), dim3((unsigned)nblk), dim3(kK1Threads), 0,
                     s, R, ld, ncol, ntiles, N, upper, snap, (const T*)cu, (const T*)v, (T*)G);
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

hipError_t launch_rank1(const Geo& g, const Snap* snap, const void* cu, const void* v, void* G,
                        hipStream_t s) {
  int nv;
  const K1Variant* tab = k1_table(g.dtype, &nv);
  hipEvent_t before, after;
  k1_take_timing(&before, &after);
  if (hipError_t er = record_event(before, s)) return note_hip(er);
  tab[k1_get_variant(g.dtype)].launch(g.R, g.ld, g.N, g.upper, snap, cu, v, G, s);
  if (hipError_t er = record_event(after, s)) return note_hip(er);
  return note_hip(hipGetLastError());
}

}  // namespace gfo
