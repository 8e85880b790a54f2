// Multi-pixel region moves: a move sets every pixel of a 2x2 region to one
// material (the paper's flipped region V with N_V = 4; Sec. IV flips 2x2-pixel
// pillars).  Regions tile the design grid; region k = by * (nx / 2) + bx, its
// pixels in row-major order.
//
// Score of (region k, material e), eqs. form4, form6-form9 at the FOM monitor
// (eq. para1), with the area-included G:
//   B = diag(b_i), b_i = k0^2 (eps_e - eps_cur_i)     (0 where pixel i is at e)
//   x = (I - G_VV B)^-1 E_V,   E'_m0 = E_m0 + G[m0, V] B x,   FOM' = |E'_m0|^2.
// The accepted move is applied as the rank-1 updates of its changed pixels, one
// after the other (exact in any order), or jointly by the rank-k step.
#include "gfo_internal.hpp"

namespace gfo {

constexpr int kRegion = 2;                       // region side
constexpr int kRegionPix = kRegion * kRegion;

__device__ __forceinline__ void region_pixels(const Geo& g, int k, int (&V)[kRegionPix]) {
  const int rx = g.nx / kRegion, by = k / rx, bx = k - by * rx;
#pragma unroll
  for (int i = 0; i < kRegionPix; ++i)
    V[i] = (by * kRegion + i / kRegion) * g.nx + bx * kRegion + i % kRegion;
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double n = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / n, (a.y * b.x - a.x * b.y) / n);
}

// One thread per region (workgroups of kScoreThreads; workgroup w covers regions
// [256 w, 256 w + 256) and leaves its best score and the lowest index within
// the tie band of that best).  The in-block entries of G are read from G, plus,
// in deferred mode, the `count` pending terms cu_s[p] v_s[q]; the diagonal comes
// from diag64 (FP64).  The 4 x 4 systems are solved in FP64 by Gaussian
// elimination with partial pivoting.
template <typename T>
__global__ __launch_bounds__(kScoreThreads) void k_score_regions(
    Geo g, int n_regions, const T* __restrict__ G, const T* __restrict__ E,
    const double2* __restrict__ diag64, const uint8_t* __restrict__ eps_idx,
    const int32_t* __restrict__ count, const T* __restrict__ CUs, const T* __restrict__ Vs,
    uint32_t mask, double tau, double* __restrict__ scores, double* __restrict__ partial,
    int* __restrict__ pfirst, int32_t* __restrict__ status) {
  __shared__ double sh[kScoreThreads / 64];
  __shared__ int shi[kScoreThreads / 64];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  Geo gr = g;                      // the region index space, for the summaries
  gr.N = n_regions;
  double F[GFO_MAX_EPS];
  double best = -INFINITY;
  bool bad = false;
  if (k < n_regions) {
    int V[kRegionPix];
    region_pixels(g, k, V);
    double2 Gvv[kRegionPix][kRegionPix], EV[kRegionPix], gm[kRegionPix];
    int cur[kRegionPix];
    const T* __restrict__ grow = G + g_off(g, g.N + g.m0, 0);
#pragma unroll
    for (int i = 0; i < kRegionPix; ++i) {
      cur[i] = eps_idx[V[i]];
      EV[i] = St<T>::to_d(E[V[i]]);
      gm[i] = St<T>::to_d(grow[V[i]]);
#pragma unroll
      for (int j = 0; j < kRegionPix; ++j)
        Gvv[i][j] = i == j ? diag64[V[i]] : St<T>::to_d(G[g_at(g, V[i], V[j])]);
    }
    const int K = count ? *count : 0;
    // terms in groups of kTermBatch: every load of a group is issued before its
    // first use (each term is an L2 round trip), the sums in term order
    constexpr int kTermBatch = 4;
    for (int s0 = 0; s0 < K; s0 += kTermBatch) {
      T cuw[kTermBatch][kRegionPix], vw[kTermBatch][kRegionPix];
#pragma unroll
      for (int u = 0; u < kTermBatch; ++u)
#pragma unroll
        for (int i = 0; i < kRegionPix; ++i)
          if (s0 + u < K) {
            cuw[u][i] = CUs[(int64_t)(s0 + u) * g.R + V[i]];
            vw[u][i] = Vs[(int64_t)(s0 + u) * g.ld + V[i]];
          }
#pragma unroll
      for (int u = 0; u < kTermBatch; ++u) {
        if (s0 + u >= K) break;
        double2 cu[kRegionPix], v[kRegionPix];
#pragma unroll
        for (int i = 0; i < kRegionPix; ++i) {
          cu[i] = St<T>::to_d(cuw[u][i]);
          v[i] = St<T>::to_d(vw[u][i]);
        }
#pragma unroll
        for (int i = 0; i < kRegionPix; ++i)
#pragma unroll
          for (int j = 0; j < kRegionPix; ++j)
            if (i != j) Gvv[i][j] = cadd(Gvv[i][j], cmul(cu[i], v[j]));
      }
    }
    const double2 Em0 = St<T>::to_d(E[g.N + g.m0]);
#pragma unroll
    for (int e = 0; e < GFO_MAX_EPS; ++e) {
      if (e >= g.n_eps) continue;
      double Fe = -INFINITY;
      bool changes = false;
#pragma unroll
      for (int i = 0; i < kRegionPix; ++i) changes |= cur[i] != e;
      if (((mask >> e) & 1u) && changes) {
        double b[kRegionPix];
#pragma unroll
        for (int i = 0; i < kRegionPix; ++i) b[i] = g.k0sq * (g.eps[e] - g.eps[cur[i]]);
        // A = I - G_VV B, augmented with E_V
        double2 A[kRegionPix][kRegionPix + 1];
#pragma unroll
        for (int i = 0; i < kRegionPix; ++i) {
#pragma unroll
          for (int j = 0; j < kRegionPix; ++j)
            A[i][j] = make_double2((i == j ? 1.0 : 0.0) - Gvv[i][j].x * b[j], -Gvv[i][j].y * b[j]);
          A[i][kRegionPix] = EV[i];
        }
#pragma unroll
        for (int c = 0; c < kRegionPix; ++c) {
          int piv = c;
          double pmax = cabs2(A[c][c]);
#pragma unroll
          for (int r = c + 1; r < kRegionPix; ++r) {
            const double m = cabs2(A[r][c]);
            if (m > pmax) {
              pmax = m;
              piv = r;
            }
          }
          if (piv != c) {
#pragma unroll
            for (int j = 0; j <= kRegionPix; ++j) {
              // swap rows c and piv without dynamic register indexing
#pragma unroll
              for (int r = c + 1; r < kRegionPix; ++r) {
                if (r == piv) {
                  const double2 t = A[c][j];
                  A[c][j] = A[r][j];
                  A[r][j] = t;
                }
              }
            }
          }
#pragma unroll
          for (int r = c + 1; r < kRegionPix; ++r) {
            const double2 f = cdiv(A[r][c], A[c][c]);
#pragma unroll
            for (int j = c; j <= kRegionPix; ++j) A[r][j] = cadd(A[r][j], cmul(make_double2(-f.x, -f.y), A[c][j]));
          }
        }
        double2 x[kRegionPix];
#pragma unroll
        for (int i = kRegionPix - 1; i >= 0; --i) {
          double2 acc = A[i][kRegionPix];
#pragma unroll
          for (int j = i + 1; j < kRegionPix; ++j) acc = cadd(acc, cmul(make_double2(-A[i][j].x, -A[i][j].y), x[j]));
          x[i] = cdiv(acc, A[i][i]);
        }
        double2 d = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < kRegionPix; ++i) d = cadd(d, cmul(gm[i], cscale(b[i], x[i])));
        Fe = cabs2(cadd(Em0, d));
        if (!isfinite(Fe)) {
          bad = true;
          Fe = -INFINITY;
        }
        best = fmax(best, Fe);
      }
      F[e] = Fe;
      scores[(int64_t)k * g.n_eps + e] = Fe;
    }
  }
  score_block_end(gr, best, k, true, F, tau, partial, pfirst, (n_regions + kScoreThreads - 1) / kScoreThreads,
                  sh, shi);
  if (bad) atomicOr(status, GFO_STATUS_NONFINITE);
}

// The greedy pick over the region scores (one wave); FOM from E at the monitor.
template <typename T>
__global__ __launch_bounds__(64) void k_region_pick(Geo g, int n_regions, const T* __restrict__ E,
                                                    const double* __restrict__ scores,
                                                    const double* __restrict__ partial,
                                                    const int* __restrict__ pfirst, double tau,
                                                    gfo_pick* __restrict__ out) {
  __shared__ double shd[1];
  __shared__ int shi[1];
  Geo gr = g;
  gr.N = n_regions;
  const double fom = cabs2(St<T>::to_d(E[g.N + g.m0]));
  const int nblk = (n_regions + kScoreThreads - 1) / kScoreThreads;
  const gfo_pick pk = greedy_pick_block(gr, fom, scores, partial, pfirst, nblk, tau, shd, shi);
  if (threadIdx.x == 0) *out = pk;
}

// The pixel moves of a region move: record i is pixel i of the region with the
// region's material, or the sentinel where the pixel already has it (or the
// region move is the sentinel).
__global__ void k_region_pixels(Geo g, const gfo_pick* __restrict__ region,
                                const uint8_t* __restrict__ eps_idx, gfo_pick* __restrict__ out) {
  const int i = threadIdx.x;
  if (i >= kRegionPix) return;
  const gfo_pick r = *region;
  gfo_pick p;
  p.pixel = -1;
  p.eps_idx = -1;
  p.fom_new = r.fom_new;
  p.dfom = r.dfom;
  const int n_regions = (g.ny / kRegion) * (g.nx / kRegion);
  if (r.pixel >= 0 && r.pixel < n_regions && r.eps_idx >= 0 && r.eps_idx < g.n_eps) {
    int V[kRegionPix];
    region_pixels(g, r.pixel, V);
    if ((int)eps_idx[V[i]] != r.eps_idx) {
      p.pixel = V[i];
      p.eps_idx = r.eps_idx;
    }
  }
  out[i] = p;
}

int region_side() { return kRegion; }

hipError_t launch_score_regions(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                                double tau, gfo_pick* out, hipStream_t s) {
  char* w = (char*)st->work;
  const int n_regions = (g.ny / kRegion) * (g.nx / kRegion);
  const int nblk = (n_regions + kScoreThreads - 1) / kScoreThreads;
  const int32_t* count = st->delay > 0 ? (const int32_t*)(w + L.dl_hdr) : nullptr;
  double* scores = (double*)(w + L.scores);
  double* partial = (double*)(w + L.partial);
  int* pfirst = (int*)(w + L.pfirst);
  if (g.dtype == GFO_C64) {
    hipLaunchKernelGGL(k_score_regions<float2>, dim3(nblk), dim3(kScoreThreads), 0, s, g, n_regions,
                       (const float2*)st->G, (const float2*)st->E, (const double2*)st->diag64,
                       (const uint8_t*)st->eps_idx, count, (const float2*)(w + L.dl_CUs),
                       (const float2*)(w + L.dl_Vs), mask, tau, scores, partial, pfirst, st->status);
    hipLaunchKernelGGL(k_region_pick<float2>, dim3(1), dim3(64), 0, s, g, n_regions,
                       (const float2*)st->E, (const double*)scores, (const double*)partial,
                       (const int*)pfirst, tau, out);
  } else {
    hipLaunchKernelGGL(k_score_regions<double2>, dim3(nblk), dim3(kScoreThreads), 0, s, g, n_regions,
                       (const double2*)st->G, (const double2*)st->E, (const double2*)st->diag64,
                       (const uint8_t*)st->eps_idx, count, (const double2*)(w + L.dl_CUs),
                       (const double2*)(w + L.dl_Vs), mask, tau, scores, partial, pfirst, st->status);
    hipLaunchKernelGGL(k_region_pick<double2>, dim3(1), dim3(64), 0, s, g, n_regions,
                       (const double2*)st->E, (const double*)scores, (const double*)partial,
                       (const int*)pfirst, tau, out);
  }
  return note_hip(hipGetLastError());
}

hipError_t launch_region_pixels(const Geo& g, const gfo_state* st, const gfo_pick* region,
                                gfo_pick* out, hipStream_t s) {
  hipLaunchKernelGGL(k_region_pixels, dim3(1), dim3(64), 0, s, g, region,
                     (const uint8_t*)st->eps_idx, out);
  return note_hip(hipGetLastError());
}

}  // namespace gfo
