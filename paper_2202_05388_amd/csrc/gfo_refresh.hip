// refresh_G: FP64 recomputation of G, E and diag64 from G0 and the flipped set.
//
// With V = {p : eps_idx[p] != background}, alpha_p = k0^2 (eps_p - eps_bg) and
// U = G0[:, V] (R x k), the discretised Dyson equation (paper eq. form2)
// restricted to V gives
//     M = (I - B_V G0[V,V])^-1 B_V = (diag(1/alpha) - G0[V,V])^-1,
//     G = G0 + U M U_D^T,   E = Einc + U M Einc[V],
// where U_D^T = G0[V, :] by reciprocity of the free-space kernel.
// Steps: flipped list -> U gather (FP64 table / direct Hankel) -> in-place
// Gauss-Jordan inverse with partial pivoting -> Z = U M (FP64 MFMA) -> E -> G = G0 + Z U_D^T
// (FP64 MFMA, G0 added in the epilogue, one rounding to the storage type) on
// the monitor rows and the symmetric design block's upper triangle, whose
// mirror gives the lower triangle when the state keeps it.
#include "gfo_internal.hpp"

namespace gfo {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 g0_kernel(double r, const Geo& g) {
  const double x = g.k0 * r, s = 0.25 * g.h * g.h;
  return make_double2(-s * y0(x), s * j0(x));
}

// G0[row, q] for a design column q; rows >= N are monitors (direct evaluation).
__device__ __forceinline__ double2 g0_entry(const Geo& g, const double2* __restrict__ table,
                                            const double* __restrict__ mon_xy, int row, int q) {
  const int iyq = q / g.nx, ixq = q - (q / g.nx) * g.nx;
  if (row < g.N) {
    const int iyr = row / g.nx, ixr = row - (row / g.nx) * g.nx;
    return table[abs(iyr - iyq) * g.nx + abs(ixr - ixq)];
  }
  const int m = row - g.N;
  const double xq = (ixq - 0.5 * (g.nx - 1)) * g.h, yq = (iyq - 0.5 * (g.ny - 1)) * g.h;
  const double dx = mon_xy[2 * m] - xq, dy = mon_xy[2 * m + 1] - yq;
  return g0_kernel(sqrt(dx * dx + dy * dy), g);
}

__device__ __forceinline__ double2 incident(const Geo& g, const double* __restrict__ mon_xy, int row) {
  double y;
  if (row < g.N) {
    y = ((row / g.nx) - 0.5 * (g.ny - 1)) * g.h;
  } else {
    y = mon_xy[2 * (row - g.N) + 1];
  }
  double s, c;
  sincos(g.k0 * y, &s, &c);
  return make_double2(c, s);
}

// ------------------------------------------------------------------ flipped list
// Single workgroup of 1024 threads: ordered compaction of {p : eps_idx[p] != bg}.
// V[N] receives the count.
__global__ __launch_bounds__(1024) void k_rf_list(Geo g, const uint8_t* __restrict__ eps_idx,
                                                  int32_t* __restrict__ V) {
  __shared__ int wsum[16];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int p0 = 0; p0 < g.N; p0 += 1024) {
    const int p = p0 + threadIdx.x;
    const int f = (p < g.N && eps_idx[p] != g.bg_idx) ? 1 : 0;
    // inclusive scan within the wave
    int x = f;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int before = base;
    for (int i = 0; i < w; ++i) before += wsum[i];
    if (f) V[before + x - 1] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int i = 0; i < 16; ++i) t += wsum[i];
      base += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) V[g.N] = base;
}

__global__ void k_rf_overflow(int32_t* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(status, GFO_STATUS_REFRESH_OVERFLOW);
}

// U[r, i] = G0[r, V_i] for i < k, 0 for k <= i < kp.  Row-major, ld = kp.
__global__ void k_rf_gather_U(Geo g, const double2* __restrict__ table,
                              const double* __restrict__ mon_xy, const int32_t* __restrict__ V,
                              int k, int kp, double2* __restrict__ U) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)g.R * kp) return;
  const int r = (int)(t / kp), i = (int)(t - (int64_t)r * kp);
  U[t] = (i < k) ? g0_entry(g, table, mon_xy, r, V[i]) : make_double2(0.0, 0.0);
}

// ------------------------------------------------------------------ Gauss-Jordan inverse
// The k x k core A = D - G0[V,V], D = diag(1 / alpha), is inverted in place,
// kp x kp with identity padding.  Step c takes as pivot p_c the row of largest
// modulus in column c among the rows not yet used (lowest row on ties), scales
// it by 1 / a[p][c] (its entry in column c becomes 1 / a[p][c]) and eliminates
// column c from every other row (their entry in column c becomes
// -a[r][c] / a[p][c]).  Rows are never swapped: after the kp steps the
// inverse is read back through the pivots, A^-1[c][p_d] = X[p_c][d].  Each step
// reads one buffer and writes the other, so no workgroup reads an entry that
// another one of the same step writes.
struct GjPart {
  double m;   // |a[r][c + 1]|^2 of the workgroup's best unused row, -1 if none
  int row;
  int pad;
};
constexpr int kGjRows = 8;   // rows per workgroup of a step

// Core A in W (row-major, ld kp) and the pivot flags cleared.
__global__ void k_rf_build_core(Geo g, const uint8_t* __restrict__ eps_idx,
                                const int32_t* __restrict__ V, const double2* __restrict__ U, int k,
                                int kp, double2* __restrict__ W, int32_t* __restrict__ used) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kp) used[t] = 0;
  if (t >= (int64_t)kp * kp) return;
  const int a = (int)(t / kp), b = (int)(t - (int64_t)a * kp);
  double2 v = make_double2(0.0, 0.0);
  if (a < k && b < k) {
    const double2 gab = U[(int64_t)V[a] * kp + b];   // G0[V_a, V_b]
    v = make_double2(-gab.x, -gab.y);
    if (a == b) {
      const double alpha = g.k0sq * (g.eps[eps_idx[V[a]]] - g.eps[g.bg_idx]);
      v.x += 1.0 / alpha;
    }
  } else if (a == b) {
    v.x = 1.0;
  }
  W[t] = v;
}

// Block-wide arg-max of (m, row), largest m and lowest row on ties; every
// thread returns the result.  256 threads.
__device__ __forceinline__ void gj_argmax(double& m, int& row) {
  __shared__ double sm[4];
  __shared__ int sr[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double om = __shfl_xor(m, o, 64);
    const int orow = __shfl_xor(row, o, 64);
    if (om > m || (om == m && orow < row)) {
      m = om;
      row = orow;
    }
  }
  if (lane == 0) {
    sm[w] = m;
    sr[w] = row;
  }
  __syncthreads();
  m = sm[0];
  row = sr[0];
#pragma unroll
  for (int q = 1; q < 4; ++q)
    if (sm[q] > m || (sm[q] == m && sr[q] < row)) {
      m = sm[q];
      row = sr[q];
    }
  __syncthreads();
}

// Step c: S -> D.  Grid: kGjRows rows (blockIdx.x) x 256 columns (blockIdx.y)
// per workgroup, one column per thread.  The pivot of column c comes from the
// previous step's candidates, one per row group (part_in, n_in), or for c = 0
// from column 0 itself.  The thread that holds column c + 1 leaves its row
// group's best unused row for the next step; the workgroup (group of p_c, 0)
// records the pivot (piv[c], used).
__global__ __launch_bounds__(256) void k_gj_step(const double2* __restrict__ S, double2* __restrict__ D,
                                                 int kp, int c, const GjPart* __restrict__ part_in,
                                                 int n_in, GjPart* __restrict__ part_out,
                                                 int32_t* __restrict__ piv, int32_t* __restrict__ used,
                                                 int32_t* __restrict__ status) {
  double best = -1.0;
  int bi = 0x7fffffff;
  if (part_in != nullptr) {
    for (int q = threadIdx.x; q < n_in; q += blockDim.x) {
      const GjPart pq = part_in[q];
      if (pq.m > best || (pq.m == best && pq.row < bi)) {
        best = pq.m;
        bi = pq.row;
      }
    }
  } else {
    for (int r = threadIdx.x; r < kp; r += blockDim.x) {
      if (used[r] != 0) continue;
      const double2 v = S[(int64_t)r * kp + c];
      double m = v.x * v.x + v.y * v.y;
      if (!(m >= 0.0)) m = 0.0;   // a NaN row stays a candidate: some row is always chosen
      if (m > best) {
        best = m;
        bi = r;
      }
    }
  }
  gj_argmax(best, bi);
  const int p = bi;
  const int r0 = blockIdx.x * kGjRows;
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    if (blockIdx.x == 0 && !(best > 0.0)) atomicOr(status, GFO_STATUS_SINGULAR);
    if (p >= r0 && p < r0 + kGjRows) {
      piv[c] = p;
      used[p] = c + 1;
    }
  }
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= kp) return;
  const double2 d = S[(int64_t)p * kp + c];
  const double n = d.x * d.x + d.y * d.y;
  const double2 inv = n > 0.0 ? make_double2(d.x / n, -d.y / n) : make_double2(1.0, 0.0);
  const double2 pc = j == c ? inv : cmul(S[(int64_t)p * kp + j], inv);
  double nb = -1.0;
  int ni = 0x7fffffff;
#pragma unroll
  for (int rr = 0; rr < kGjRows; ++rr) {
    const int r = r0 + rr;
    if (r < kp) {
      double2 out = pc;
      if (r != p) {
        const double2 fr = S[(int64_t)r * kp + c];
        const double2 v = j == c ? make_double2(0.0, 0.0) : S[(int64_t)r * kp + j];
        out = make_double2(v.x - (fr.x * pc.x - fr.y * pc.y), v.y - (fr.x * pc.y + fr.y * pc.x));
      }
      D[(int64_t)r * kp + j] = out;
      // a candidate pivot of column c + 1: not p, not used before this step
      if (j == c + 1 && r != p && used[r] == 0) {
        double m = out.x * out.x + out.y * out.y;
        if (!(m >= 0.0)) m = 0.0;
        if (m > nb) {   // rows in increasing order: the lowest row wins ties
          nb = m;
          ni = r;
        }
      }
    }
  }
  if (j == c + 1) part_out[blockIdx.x] = GjPart{nb, ni, 0};
}

// M = A^-1 from the in-place result X: M[c][p_d] = X[p_c][d].
__global__ void k_gj_unpermute(const double2* __restrict__ X, double2* __restrict__ M,
                               const int32_t* __restrict__ piv, int kp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)kp * kp) return;
  const int c = (int)(t / kp), d = (int)(t - (int64_t)c * kp);
  M[(int64_t)c * kp + piv[d]] = X[(int64_t)piv[c] * kp + d];
}

// Blocked form (k > 64): panels of kGjPanel columns.  A panel's columns are
// copied to a k x kGjPanel buffer and its steps run there (the same pivot rule,
// the same updates restricted to the panel's columns, two buffers); the
// panel's transformation T = prod of its steps then reaches every other
// column j at once: X'[:, j] = X[:, j] + (T[:, P] - I[:, P]) X[P, j], P the
// panel's pivot rows, whose columns T[:, P] the panel buffer now holds (column
// c for pivot p_c).  That is a rank-kGjPanel FP64 product on the matrix cores,
// its pivot rows read from a copy taken before; in the pivot rows the -1
// cancels the old value.  used[r] = c + 1 records the column r pivoted.
constexpr int kGjPanel = 32;

__global__ void k_gj_panel_copy(const double2* __restrict__ X, double2* __restrict__ Pn, int kp, int c0,
                                int qn) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)kp * kGjPanel) return;
  const int r = (int)(t / kGjPanel), i = (int)(t - (int64_t)r * kGjPanel);
  if (i < qn) Pn[t] = X[(int64_t)r * kp + c0 + i];
}

// Panel step c (local column ci = c - c0): S -> D, 8 rows x 32 columns per
// workgroup; the pivot from the previous step's candidates (part_in) or, for
// the panel's first column, from a scan of the unused rows.
__global__ __launch_bounds__(256) void k_gj_panel_step(const double2* __restrict__ S, double2* __restrict__ D,
                                                       int kp, int c0, int qn, int c,
                                                       const GjPart* __restrict__ part_in, int n_in,
                                                       GjPart* __restrict__ part_out, int32_t* __restrict__ piv,
                                                       int32_t* __restrict__ used, int32_t* __restrict__ status) {
  const int ci = c - c0;
  double best = -1.0;
  int bi = 0x7fffffff;
  if (part_in != nullptr) {
    for (int q = threadIdx.x; q < n_in; q += blockDim.x) {
      const GjPart pq = part_in[q];
      if (pq.m > best || (pq.m == best && pq.row < bi)) {
        best = pq.m;
        bi = pq.row;
      }
    }
  } else {
    for (int r = threadIdx.x; r < kp; r += blockDim.x) {
      if (used[r] != 0) continue;
      const double2 v = S[(int64_t)r * kGjPanel + ci];
      double m = v.x * v.x + v.y * v.y;
      if (!(m >= 0.0)) m = 0.0;
      if (m > best) {
        best = m;
        bi = r;
      }
    }
  }
  gj_argmax(best, bi);
  const int p = bi;
  const int r0 = blockIdx.x * kGjRows;
  if (threadIdx.x == 0) {
    if (blockIdx.x == 0 && !(best > 0.0)) atomicOr(status, GFO_STATUS_SINGULAR);
    if (p >= r0 && p < r0 + kGjRows) {
      piv[c] = p;
      used[p] = c + 1;
    }
  }
  const int r = r0 + (int)(threadIdx.x >> 5), i = (int)(threadIdx.x & 31);
  double nb = -1.0;
  int ni = 0x7fffffff;
  if (r < kp && i < qn) {
    const double2 d = S[(int64_t)p * kGjPanel + ci];
    const double n = d.x * d.x + d.y * d.y;
    const double2 inv = n > 0.0 ? make_double2(d.x / n, -d.y / n) : make_double2(1.0, 0.0);
    const double2 pc = i == ci ? inv : cmul(S[(int64_t)p * kGjPanel + i], inv);
    double2 out = pc;
    if (r != p) {
      const double2 fr = S[(int64_t)r * kGjPanel + ci];
      const double2 v = i == ci ? make_double2(0.0, 0.0) : S[(int64_t)r * kGjPanel + i];
      out = make_double2(v.x - (fr.x * pc.x - fr.y * pc.y), v.y - (fr.x * pc.y + fr.y * pc.x));
    }
    D[(int64_t)r * kGjPanel + i] = out;
    if (i == ci + 1 && r != p && used[r] == 0) {
      double m = out.x * out.x + out.y * out.y;
      if (!(m >= 0.0)) m = 0.0;
      nb = m;
      ni = r;
    }
  }
  gj_argmax(nb, ni);
  if (threadIdx.x == 0) part_out[blockIdx.x] = GjPart{nb, ni, 0};
}

// The pivot rows of the panel before it: Prow[i][j] = X[p_(c0 + i)][j].
__global__ void k_gj_pivot_rows(const double2* __restrict__ X, double2* __restrict__ Prow,
                                const int32_t* __restrict__ piv, int kp, int c0, int qn) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)qn * kp) return;
  const int i = (int)(t / kp), j = (int)(t - (int64_t)i * kp);
  Prow[t] = X[(int64_t)piv[c0 + i] * kp + j];
}

// Epilogue of the panel's product v = (T[:, P] X[P, :])[m][n]: the panel's
// columns take T[:, P]; a pivot row of the panel takes v; every other entry adds v.
struct EpiGJ {
  double2* X;
  const double2* Pn;
  const int32_t* used;
  int kp, c0, qn;
  __device__ void operator()(int m, int n, double2 v) const {
    double2* x = X + (int64_t)m * kp + n;
    if (n >= c0 && n < c0 + qn) {
      *x = Pn[(int64_t)m * kGjPanel + (n - c0)];
    } else {
      const int u = used[m];
      *x = (u > c0 && u <= c0 + qn) ? v : cadd(*x, v);
    }
  }
};

// ------------------------------------------------------------------ FP64 MFMA complex GEMM
// C(m, n) = sum_k A(m, k) B(k, n), complex FP64, A row-major (lda).
// B(k, n) = Bp[k * ldb + n] (BT = false) or Bp[n * ldb + k] (BT = true).
// Workgroup 256 threads = 4 waves, tile 64 x 64; each wave 32 x 32 = 2 x 2
// v_mfma_f64_16x16x4 tiles, with separate real and imaginary accumulators:
//   re += Ar Br - Ai Bi,  im += Ar Bi + Ai Br.
// Operand layout of the 16x16x4 FP64 instruction (one value per lane):
//   A(i, k): i = lane % 16, k = lane / 16;  B(k, j): j = lane % 16, k = lane / 16;
//   D(i, j): j = lane % 16, i = lane / 16 + 4 * element  (checked on gfx950).
struct EpiStoreZ {
  double2* Z;
  int64_t ldz;
  __device__ void operator()(int m, int n, double2 v) const { Z[(int64_t)m * ldz + n] = v; }
};

template <typename T>
struct EpiG0 {
  Geo g;
  const double2* table;
  const double* mon_xy;
  T* G;
  double2* diag64;
  __device__ void operator()(int m, int n, double2 v) const {
    // band-packed storage holds no entry left of a design row's band
    if (g.packed && m < g.N && n < (m & ~63)) return;
    const double2 g0 = g0_entry(g, table, mon_xy, m, n);
    const double2 val = make_double2(g0.x + v.x, g0.y + v.y);
    G[g_off(g, m, n)] = St<T>::from_d(val);
    if (m == n) diag64[m] = val;
  }
};

struct EpiAddG {
  Geo g;
  double2* G;
  __device__ void operator()(int m, int n, double2 v) const {
    if (g.packed && m < g.N && n < (m & ~63)) return;
    double2* p = G + g_off(g, m, n);
    *p = cadd(*p, v);
  }
};

// A(m, k) = A[m * lda + k], or A[k * lda + m] when AT; K is clamped to *kdev when given.
// skip_below > 0: tiles wholly below the diagonal within rows < skip_below are
// not computed (deferred mode keeps the design block's upper triangle only);
// the launch is then a 1-D grid of the other tiles only (ut_group).
// Four waves per SIMD requested: the accumulators then live in ordinary vector
// registers and every instantiation fits 4-5 waves without spilling (left to
// itself the compiler put them in accumulation registers at 2-3 waves, and the
// matrix instructions waited on their operand loads).
template <bool AT, bool BT, typename Epi>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_zgemm_f64(int M, int N, int K, const double2* __restrict__ A,
                                                   int64_t lda, const double2* __restrict__ B,
                                                   int64_t ldb, const int32_t* __restrict__ kdev,
                                                   Epi epi, int skip_below) {
  int by = (int)blockIdx.y, bx = (int)blockIdx.x;
  if (skip_below > 0) ut_group(blockIdx.x, (N + 63) / 64, skip_below / 64, 64, 64, by, bx);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = by * 64 + (w >> 1) * 32;
  const int n0 = bx * 64 + (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 re[2][2], im[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      re[t][u] = (f64x4){0.0, 0.0, 0.0, 0.0};
      im[t][u] = (f64x4){0.0, 0.0, 0.0, 0.0};
    }
  if (kdev != nullptr) K = min(K, *kdev);
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int kk = k0 + lk;
    double2 a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int row = m0 + 16 * t + li;
      if (row < M && kk < K)
        a[t] = AT ? A[(int64_t)kk * lda + row] : A[(int64_t)row * lda + kk];
      else
        a[t] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int col = n0 + 16 * u + li;
      if (col < N && kk < K)
        b[u] = BT ? B[(int64_t)col * ldb + kk] : B[(int64_t)kk * ldb + col];
      else
        b[u] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        re[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].x, b[u].x, re[t][u], 0, 0, 0);
        re[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[t].y, b[u].y, re[t][u], 0, 0, 0);
        im[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].x, b[u].y, im[t][u], 0, 0, 0);
        im[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].y, b[u].x, im[t][u], 0, 0, 0);
      }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + 16 * t + lk + 4 * e;
        const int col = n0 + 16 * u + li;
        if (row < M && col < N) epi(row, col, make_double2(re[t][u][e], im[t][u][e]));
      }
}

// The same product with a 128 x 128 output tile per workgroup of 512 threads
// (8 waves in 2 x 4, each 64 x 32 = 4 x 2 tiles of the 16x16x4 instruction),
// for the refresh, whose k is the flipped set (hundreds to thousands).  The
// operands pass through LDS in chunks of 8 k with two buffers: the next chunk
// is loaded into registers while the current one is multiplied, and a wave
// waits on global memory only when it stores that chunk to LDS, 64 matrix
// instructions later.  Each operand element is fetched once per workgroup
// (1/32 byte per flop, against 1/8 for the 64 x 64 tile, whose waves each load
// their own rows and columns).  It holds one workgroup per compute unit (two
// waves per SIMD), so its epilogue does not overlap other tiles' products: the
// 64 x 64 kernel stays the faster one for the flush's k <= 128, whose
// epilogue reads and writes G.
// Every accumulator takes the same instructions on the same operands in the
// same order as in k_zgemm_f64, and the epilogue covers the same entries (the
// 64 x 64 tiles wholly below the diagonal within rows < skip_below are left
// alone), so the two kernels give bitwise equal results.
constexpr int kZgT = 128, kZgKC = 8, kZgPitch = kZgT + 1;  // pitch: one pad entry per k row

template <bool AT, bool BT, typename Epi>
__global__ __launch_bounds__(512) void k_zgemm_f64_t128(int M, int N, int K, const double2* __restrict__ A,
                                                        int64_t lda, const double2* __restrict__ B,
                                                        int64_t ldb, const int32_t* __restrict__ kdev,
                                                        Epi epi, int skip_below) {
  int by = (int)blockIdx.y, bx = (int)blockIdx.x;
  if (skip_below > 0) ut_group(blockIdx.x, (N + kZgT - 1) / kZgT, skip_below / kZgT, kZgT, kZgT, by, bx);
  __shared__ double2 As[2][kZgKC][kZgPitch], Bs[2][kZgKC][kZgPitch];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int tm0 = by * kZgT, tn0 = bx * kZgT;
  const int wm = (w >> 2) * 64, wn = (w & 3) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // the wave's rows and columns lie in one 64 x 64 tile; a skipped one idles
  const int ty = (tm0 + wm) >> 6, tx = (tn0 + wn) >> 6;
  const bool idle = skip_below > 0 && ty > tx && ((int64_t)ty + 1) * 64 <= skip_below;
  if (kdev != nullptr) K = min(K, *kdev);
  f64x4 re[4][2], im[4][2];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      re[t][u] = (f64x4){0.0, 0.0, 0.0, 0.0};
      im[t][u] = (f64x4){0.0, 0.0, 0.0, 0.0};
    }
  // staging: thread tid moves elements tid and tid + 512 of each 128 x 8 chunk,
  // consecutive threads along the operand's contiguous index
  auto a_pos = [](int e, int& r, int& kk) {
    if (AT) { r = e & 127; kk = e >> 7; } else { r = e >> 3; kk = e & 7; }
  };
  auto b_pos = [](int e, int& c, int& kk) {
    if (BT) { c = e >> 3; kk = e & 7; } else { c = e & 127; kk = e >> 7; }
  };
  double2 pa[2], pb[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int r, c, ka, kb;
      a_pos(tid + 512 * i, r, ka);
      b_pos(tid + 512 * i, c, kb);
      const int row = tm0 + r, col = tn0 + c;
      ka += k0;
      kb += k0;
      pa[i] = row < M && ka < K ? (AT ? A[(int64_t)ka * lda + row] : A[(int64_t)row * lda + ka])
                                : make_double2(0.0, 0.0);
      pb[i] = col < N && kb < K ? (BT ? B[(int64_t)col * ldb + kb] : B[(int64_t)kb * ldb + col])
                                : make_double2(0.0, 0.0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int r, c, ka, kb;
      a_pos(tid + 512 * i, r, ka);
      b_pos(tid + 512 * i, c, kb);
      As[buf][ka][r] = pa[i];
      Bs[buf][kb][c] = pb[i];
    }
  };
  const int nch = (K + kZgKC - 1) / kZgKC;
  if (nch > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) load((ch + 1) * kZgKC);
    if (!idle) {
#pragma unroll
      for (int st = 0; st < kZgKC / 4; ++st) {
        if (ch * kZgKC + 4 * st >= K) break;
        double2 a[4], b[2];
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = As[buf][4 * st + lk][wm + 16 * t + li];
#pragma unroll
        for (int u = 0; u < 2; ++u) b[u] = Bs[buf][4 * st + lk][wn + 16 * u + li];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            re[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].x, b[u].x, re[t][u], 0, 0, 0);
            re[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[t].y, b[u].y, re[t][u], 0, 0, 0);
            im[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].x, b[u].y, im[t][u], 0, 0, 0);
            im[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].y, b[u].x, im[t][u], 0, 0, 0);
          }
      }
    }
    if (ch + 1 < nch) store(buf ^ 1);
    __syncthreads();
  }
  if (idle) return;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = tm0 + wm + 16 * t + lk + 4 * e;
        const int col = tn0 + wn + 16 * u + li;
        if (row < M && col < N) epi(row, col, make_double2(re[t][u][e], im[t][u][e]));
      }
}

// x = M Einc[V] (k-vector), then E[r] = Einc[r] + sum_i U[r, i] x_i.
__global__ void k_rf_xE(Geo g, const double* __restrict__ mon_xy, const int32_t* __restrict__ V,
                        const double2* __restrict__ M, int k, int kp, double2* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kp) return;
  double2 s = make_double2(0.0, 0.0);
  if (i < k)
    for (int j = 0; j < k; ++j)
      s = cadd(s, cmul(M[(int64_t)i * kp + j], incident(g, mon_xy, V[j])));
  x[i] = s;
}

template <typename T>
__global__ void k_rf_field(Geo g, const double* __restrict__ mon_xy, const double2* __restrict__ U,
                           const double2* __restrict__ x, int k, int kp, T* __restrict__ E) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.R) return;
  double2 s = incident(g, mon_xy, r);
  for (int i = 0; i < k; ++i) s = cadd(s, cmul(U[(int64_t)r * kp + i], x[i]));
  E[r] = St<T>::from_d(s);
}

// Flipped list V (in the workspace) and its length k, read back to the host
// (one stream synchronisation).  Changes nothing else.
int launch_refresh_count(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s,
                         int32_t* k) {
  int32_t* V = (int32_t*)((char*)st->work + L.rf_V);
  hipLaunchKernelGGL(k_rf_list, dim3(1), dim3(1024), 0, s, g, (const uint8_t*)st->eps_idx, V);
  *k = 0;
  if (note_hip(hipMemcpyAsync(k, V + g.N, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      note_hip(hipStreamSynchronize(s)) != hipSuccess)
    return GFO_EHIP;
  return GFO_OK;
}

hipError_t launch_refresh_overflow(gfo_state* st, hipStream_t s) {
  hipLaunchKernelGGL(k_rf_overflow, dim3(1), dim3(64), 0, s, st->status);
  return note_hip(hipGetLastError());
}

template <typename T>
static int refresh_typed(const Geo& g, gfo_state* st, const Layout& L, int32_t k, hipStream_t s) {
  char* w = (char*)st->work;
  const double2* table = (const double2*)(w + L.table);
  const double* mon = (const double*)(w + L.mon_xy);
  int32_t* V = (int32_t*)(w + L.rf_V);
  double2* U = (double2*)(w + L.rf_U);
  double2* Z = (double2*)(w + L.rf_Z);
  double2* x = (double2*)(w + L.rf_x);
  const int kp = (k + 3) / 4 * 4;
  double2* M = nullptr;
  if (kp > 0) {
    const int64_t nu = (int64_t)g.R * kp;
    hipLaunchKernelGGL(k_rf_gather_U, dim3((unsigned)((nu + 255) / 256)), dim3(256), 0, s, g, table,
                       mon, (const int32_t*)V, k, kp, U);
    // two kp x kp buffers in the 2 kp^2 entries of rf_A; in rf_piv (16 kp + 64
    // bytes): the per-workgroup candidates of two steps, the pivots, the flags
    const int nb = (kp + kGjRows - 1) / kGjRows;
    double2* W[2] = {(double2*)(w + L.rf_A), (double2*)(w + L.rf_A) + (int64_t)kp * kp};
    GjPart* part[2] = {(GjPart*)(w + L.rf_piv), (GjPart*)(w + L.rf_piv) + nb};
    int32_t* piv = (int32_t*)(part[1] + nb);
    int32_t* used = piv + kp;
    const int64_t na = (int64_t)kp * kp;
    hipLaunchKernelGGL(k_rf_build_core, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, g,
                       (const uint8_t*)st->eps_idx, (const int32_t*)V, (const double2*)U, k, kp, W[0],
                       used);
    const double2* X = nullptr;   // the in-place result
    if (kp > 2 * kGjPanel && g.R >= 3 * kGjPanel) {
      // blocked: the panel buffers and the pivot rows' copy in Z's workspace
      // (R x kp entries, free until Z = U M), X in place in W[0]
      double2* Pn[2] = {Z, Z + (int64_t)kp * kGjPanel};
      double2* Prow = Z + 2 * (int64_t)kp * kGjPanel;
      const unsigned np = (unsigned)(((int64_t)kp * kGjPanel + 255) / 256);
      for (int c0 = 0; c0 < kp; c0 += kGjPanel) {
        const int qn = min(kGjPanel, kp - c0);
        hipLaunchKernelGGL(k_gj_panel_copy, dim3(np), dim3(256), 0, s, (const double2*)W[0], Pn[0], kp, c0,
                           qn);
        for (int l = 0; l < qn; ++l)
          hipLaunchKernelGGL(k_gj_panel_step, dim3((unsigned)nb), dim3(256), 0, s, (const double2*)Pn[l & 1],
                             Pn[(l + 1) & 1], kp, c0, qn, c0 + l,
                             l == 0 ? (const GjPart*)nullptr : (const GjPart*)part[(l + 1) & 1], nb,
                             part[l & 1], piv, used, st->status);
        hipLaunchKernelGGL(k_gj_pivot_rows, dim3((unsigned)(((int64_t)qn * kp + 255) / 256)), dim3(256), 0, s,
                           (const double2*)W[0], Prow, (const int32_t*)piv, kp, c0, qn);
        EpiGJ eg{W[0], Pn[qn & 1], used, kp, c0, qn};
        hipLaunchKernelGGL((k_zgemm_f64<false, false, EpiGJ>), dim3((kp + 63) / 64, (kp + 63) / 64), dim3(256),
                           0, s, kp, kp, qn, (const double2*)Pn[qn & 1], (int64_t)kGjPanel,
                           (const double2*)Prow, (int64_t)kp, (const int32_t*)nullptr, eg, 0);
      }
      X = W[0];
      M = W[1];
    } else {
      const dim3 gj_grid((unsigned)nb, (unsigned)((kp + 255) / 256));
      for (int c = 0; c < kp; ++c)
        hipLaunchKernelGGL(k_gj_step, gj_grid, dim3(256), 0, s, (const double2*)W[c & 1],
                           W[(c + 1) & 1], kp, c, c == 0 ? (const GjPart*)nullptr : (const GjPart*)part[(c + 1) & 1],
                           nb, part[c & 1], piv, used, st->status);
      // after kp steps the in-place result is in W[kp & 1]; M goes to the other
      X = W[kp & 1];
      M = W[(kp + 1) & 1];
    }
    hipLaunchKernelGGL(k_gj_unpermute, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, X, M,
                       (const int32_t*)piv, kp);
    // Z = U M
    EpiStoreZ ez{Z, kp};
    hipLaunchKernelGGL((k_zgemm_f64_t128<false, false, EpiStoreZ>),
                       dim3((kp + kZgT - 1) / kZgT, (g.R + kZgT - 1) / kZgT), dim3(512), 0, s, g.R, kp, kp,
                       (const double2*)U, (int64_t)kp, (const double2*)M, (int64_t)kp,
                       (const int32_t*)nullptr, ez, 0);
    hipLaunchKernelGGL(k_rf_xE, dim3((kp + 255) / 256), dim3(256), 0, s, g, mon, (const int32_t*)V,
                       (const double2*)M, k, kp, x);
  }
  hipLaunchKernelGGL(k_rf_field<T>, dim3((g.R + 255) / 256), dim3(256), 0, s, g, mon,
                     (const double2*)U, (const double2*)x, k, kp, (T*)st->E);
  // G = G0 + Z U_D^T over the N design columns (padding columns stay zero):
  // the monitor rows whole and the design block on and above its diagonal (the
  // block is symmetric); when the caller keeps the whole block, its lower
  // triangle is then the mirror of the upper one (half the product's work)
  EpiG0<T> eg{g, table, mon, (T*)st->G, (double2*)st->diag64};
  const int ty = (g.R + kZgT - 1) / kZgT, tx = (g.N + kZgT - 1) / kZgT;
  hipLaunchKernelGGL((k_zgemm_f64_t128<false, true, EpiG0<T>>),
                     dim3((unsigned)ut_group_count(ty, tx, g.N / kZgT, kZgT, kZgT)), dim3(512), 0, s, g.R, g.N, kp,
                     (const double2*)Z, (int64_t)kp,
                     (const double2*)U, (int64_t)kp, (const int32_t*)nullptr, eg, g.N);
  if (note_hip(hipGetLastError()) != hipSuccess) return GFO_EHIP;
  if (!g.upper && launch_sync_lower(g, st, s) != hipSuccess) return GFO_EHIP;   // dense storage
  return GFO_OK;
}

// Deferred-mode flush for complex128 storage: G[r, 0:N] += CU V^T over the
// `count` pending terms (FP64 matrix cores), for the monitor rows and the design
// block's tiles on and above its diagonal (the caller marks the lower triangle
// out of date).
hipError_t launch_zgemm_update_f64(const Geo& g, const int32_t* count, const double2* CU,
                                   const double2* V, double2* G, hipStream_t s) {
  // slot-major terms: A(m, k) = CU[k * R + m], B(k, n) = V[k * ld + n]; all R
  // rows (the design block and the monitor rows; the FOM monitor's terms are
  // zeros)
  EpiAddG ep{g, G};
  const int ty = (g.R + 63) / 64, tx = (g.N + 63) / 64;
  hipLaunchKernelGGL((k_zgemm_f64<true, false, EpiAddG>), dim3((unsigned)ut_group_count(ty, tx, g.N / 64, 64, 64)),
                     dim3(256), 0, s, g.R, g.N, GFO_MAX_DELAY, CU, (int64_t)g.R, V, g.ld, count, ep, g.N);
  return note_hip(hipGetLastError());
}

int launch_refresh(const Geo& g, gfo_state* st, const Layout& L, int32_t k, hipStream_t s) {
  if (g.dtype == GFO_C64) return refresh_typed<float2>(g, st, L, k, s);
  return refresh_typed<double2>(g, st, L, k, s);
}

}  // namespace gfo
