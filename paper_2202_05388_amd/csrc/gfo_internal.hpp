// Internal definitions shared by the libgfo HIP sources: the kernel parameter
// block, FP64 complex helpers, storage-type traits and the workspace layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/gfo.h"

namespace gfo {

// Geometry and material data passed by value to every kernel.
struct Geo {
  int ny, nx, nmon, N, R;
  int64_t ld;
  double k0, k0sq, h;
  double eps[GFO_MAX_EPS];
  int n_eps, bg_idx, m0;
  int dtype;
};

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
};

constexpr int kScoreThreads = 256;
constexpr int kScoreMaxBlocks = 1024;
constexpr int kSelectThreads = 1024;

// ------------------------------------------------------------------ workspace layout
struct Layout {
  size_t table;     // ny*nx double2: G0 over non-negative pixel offsets
  size_t mon_xy;    // 2*nmon double
  size_t scores;    // N*n_eps double
  size_t partial;   // kScoreMaxBlocks double
  size_t picks;     // GFO_MAX_RANK_K gfo_pick (internal rank-k scratch)
  size_t snap;      // Snap
  size_t cu;        // R x 16 B: c * G[:, j] (storage type)
  size_t v;         // ld x 16 B: G[j, :] (storage type), zero padded to ld
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
  size_t dl_CU;     // R x GFO_MAX_DELAY x 16 B: c * G[:, j] of each pending move, element-major
  size_t dl_V;      // ld x GFO_MAX_DELAY x 16 B: G[j, :] of each pending move, element-major
  size_t dl_CUs;    // the same terms slot-major: GFO_MAX_DELAY x R x 16 B
  size_t dl_Vs;     // slot-major: GFO_MAX_DELAY x ld x 16 B
  // refresh
  // (kp = kmax rounded up to a multiple of 4)
  size_t rf_V;      // N + 1 int32: flipped list, then its length
  size_t rf_U;      // R x kp double2: G0[:, V]
  size_t rf_A;      // kp x 2kp double2: Gauss-Jordan on [diag(1/alpha) - G0[V,V] | I]
  size_t rf_piv;    // kp double2: pivot column of the current Gauss-Jordan step
  size_t rf_Z;      // R x kp double2: G0[:, V] M
  size_t rf_x;      // kp double2: M Einc[V]
  size_t total;
};

Layout make_layout(const gfo_problem* p, int64_t ld, int32_t kmax);
Geo make_geo(const gfo_problem* p, int64_t ld);
int validate_problem(const gfo_problem* p);
int find_bg(const gfo_problem* p);

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------------ launchers
hipError_t launch_init(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s);
hipError_t launch_score(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                        double tau, int topk, int spacing, gfo_pick* out, hipStream_t s);
hipError_t launch_apply(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                        hipStream_t s);
hipError_t launch_rank_k(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* picks,
                         int k, int precision, hipStream_t s);
int launch_refresh(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s);
hipError_t launch_flush(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s);
template <typename T>
hipError_t launch_apply_deferred(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                                 hipStream_t s);
hipError_t launch_zgemm_update_f64(const Geo& g, const int32_t* count, const double2* CU,
                                   const double2* V, double2* G, hipStream_t s);
hipError_t launch_dl_reset(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s);

// K1 variant selection (autotuner); returns number of variants
int k1_variant_count(int dtype);
const char* k1_variant_name(int dtype, int idx);
int k1_set_variant(int dtype, int idx);
int k1_get_variant(int dtype);
void k1_time_next(hipEvent_t before, hipEvent_t after);
void k1_take_timing(hipEvent_t* before, hipEvent_t* after);   // consumes the pending pair
int flush_variant_count();
const char* flush_variant_name(int idx);
int flush_set_variant(int idx);
int flush_get_variant();

}  // namespace gfo
