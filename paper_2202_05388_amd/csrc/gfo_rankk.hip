// apply_flips_rank_k: joint update of s <= 32 accepted moves (paper eqs.
// form10-form14 with V = the s pixels, i.e. the Woodbury identity):
//   M = (I - B_S G[S,S])^-1 B_S            (s x s, FP64, Gauss-Jordan in LDS)
//   G += G[:, S] (M G[S, :]) = U W         (rank-s, matrix cores)
//   E += U (M E[S]),  diag64 += diag(U W) (FP64).
// The R x N product is done as two real GEMMs with a shared A operand:
//   A = [Re U | Im U]  (R x 2KP),  B_re = [Re W ; -Im W],  B_im = [Im W ; Re W],
//   Re(UW) = A B_re,   Im(UW) = A B_im,
// with FP32 (v_mfma_f32_32x32x2_f32) or BF16 (v_mfma_f32_32x32x16_bf16)
// inputs and FP32 accumulation into the complex64 G tile.
#include "gfo_internal.hpp"

#include <atomic>

namespace gfo {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int KR = GFO_MAX_RANK_K;   // storage stride of the rank dimension

struct RkHdr {
  int32_t s;
  int32_t kp;
  int32_t pad[2];
  int32_t S[KR];
  int32_t e_new[KR];
  double alpha[KR];
  double2 y[KR];      // M E[S]
};
static_assert(sizeof(RkHdr) <= 4096, "rank-k header exceeds its workspace slot");

// ------------------------------------------------------------------ RK1: prepare
template <typename T>
__global__ __launch_bounds__(256) void k_rk_prepare(Geo g, const gfo_pick* __restrict__ picks,
                                                    int k, const T* __restrict__ G,
                                                    const T* __restrict__ E,
                                                    const double2* __restrict__ diag64,
                                                    uint8_t* __restrict__ eps_idx,
                                                    int32_t* __restrict__ flips, int flip_cap,
                                                    int32_t* __restrict__ n_flips,
                                                    int32_t* __restrict__ status,
                                                    RkHdr* __restrict__ hdr,
                                                    double2* __restrict__ Mout) {
  __shared__ double2 aug[KR][2 * KR + 1];
  __shared__ double2 fcol[KR];
  __shared__ int S[KR], en[KR];
  __shared__ double al[KR];
  __shared__ int ns, piv, bad;
  if (threadIdx.x == 0) {
    int s = 0;
    for (int t = 0; t < k; ++t) {
      const gfo_pick pk = picks[t];
      const int j = pk.pixel, e = pk.eps_idx;
      if (j < 0 || j >= g.N || e < 0 || e >= g.n_eps || e == (int)eps_idx[j]) continue;
      bool dup = false;
      for (int q = 0; q < s; ++q) dup |= (S[q] == j);
      if (dup) continue;
      S[s] = j;
      en[s] = e;
      al[s] = g.k0sq * (g.eps[e] - g.eps[eps_idx[j]]);
      ++s;
    }
    ns = s;
    bad = 0;
  }
  __syncthreads();
  const int s = ns;
  // [I - B_S G_SS | B_S]
  for (int idx = threadIdx.x; idx < s * 2 * s; idx += blockDim.x) {
    const int a = idx / (2 * s), b = idx - (idx / (2 * s)) * 2 * s;
    double2 v;
    if (b < s) {
      const double2 gab = (a == b) ? diag64[S[a]] : St<T>::to_d(G[g_at(g, S[a], S[b])]);
      v = make_double2((a == b ? 1.0 : 0.0) - al[a] * gab.x, -al[a] * gab.y);
    } else {
      v = make_double2(b - s == a ? al[a] : 0.0, 0.0);
    }
    aug[a][b] = v;
  }
  __syncthreads();
  for (int c = 0; c < s; ++c) {
    if (threadIdx.x == 0) {
      int p = c;
      double best = cabs2(aug[c][c]);
      for (int r = c + 1; r < s; ++r) {
        const double m = cabs2(aug[r][c]);
        if (m > best) {
          best = m;
          p = r;
        }
      }
      if (!(best > 1e-24)) bad = 1;
      piv = p;
    }
    __syncthreads();
    const int p = piv;
    if (p != c)
      for (int j = threadIdx.x; j < 2 * s; j += blockDim.x) {
        const double2 t = aug[c][j];
        aug[c][j] = aug[p][j];
        aug[p][j] = t;
      }
    __syncthreads();
    const double2 inv = rdiv(1.0, aug[c][c]);
    __syncthreads();
    for (int j = threadIdx.x; j < 2 * s; j += blockDim.x) aug[c][j] = cmul(aug[c][j], inv);
    for (int r = threadIdx.x; r < s; r += blockDim.x) fcol[r] = aug[r][c];
    __syncthreads();
    for (int idx = threadIdx.x; idx < s * 2 * s; idx += blockDim.x) {
      const int r = idx / (2 * s), j = idx - (idx / (2 * s)) * 2 * s;
      if (r != c) {
        const double2 f = fcol[r];
        const double2 pc = aug[c][j];
        aug[r][j] = make_double2(aug[r][j].x - (f.x * pc.x - f.y * pc.y),
                                 aug[r][j].y - (f.x * pc.y + f.y * pc.x));
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && bad) atomicOr(status, GFO_STATUS_SINGULAR);
  const int sv = bad ? 0 : s;
  for (int idx = threadIdx.x; idx < KR * KR; idx += blockDim.x) {
    const int a = idx / KR, b = idx - (idx / KR) * KR;
    Mout[idx] = (a < sv && b < sv) ? aug[a][s + b] : make_double2(0.0, 0.0);
  }
  if (threadIdx.x < KR) {
    const int a = threadIdx.x;
    double2 y = make_double2(0.0, 0.0);
    if (a < sv)
      for (int b = 0; b < sv; ++b) y = cadd(y, cmul(aug[a][s + b], St<T>::to_d(E[S[b]])));
    hdr->y[a] = y;
    hdr->S[a] = a < sv ? S[a] : 0;
    hdr->e_new[a] = a < sv ? en[a] : 0;
    hdr->alpha[a] = a < sv ? al[a] : 0.0;
  }
  if (threadIdx.x == 0) {
    hdr->s = sv;
    hdr->kp = sv <= 16 ? 16 : 32;
    int n = *n_flips;
    for (int a = 0; a < sv; ++a) {
      eps_idx[S[a]] = (uint8_t)en[a];
      if (n < flip_cap) {
        flips[2 * n] = S[a];
        flips[2 * n + 1] = en[a];
      } else {
        atomicOr(status, GFO_STATUS_HISTORY_FULL);
      }
      ++n;
    }
    *n_flips = n;
  }
}

// ------------------------------------------------------------------ RK2: rows (U = G[:, S])
// One thread per row in 64-thread workgroups (a few hundred workgroups at
// 128 x 128); the s <= 32 loads of a row are unrolled, so all of them are in
// flight together.  Writes U64 (R x KR, FP64, for the diagonal in RK3) and the
// A operand row-major [r][kappa], kappa < KP: Re U, kappa >= KP: Im U, in FP32
// (Af) or BF16 (Abf), with 16-byte stores; E[r] += U[r, :] y.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
template <typename T>
__global__ __launch_bounds__(64) void k_rk_rows(Geo g, const RkHdr* __restrict__ hdr,
                                                const T* __restrict__ G,
                                                const double2* __restrict__ diag64,
                                                T* __restrict__ E, double2* __restrict__ U64,
                                                float* __restrict__ Af, __bf16* __restrict__ Abf,
                                                int bf16) {
  __shared__ int S[KR];
  __shared__ double2 y[KR];
  const int s = hdr->s;
  if (s == 0) return;
  const int KP = hdr->kp;
  if (threadIdx.x < KR) {
    S[threadIdx.x] = hdr->S[threadIdx.x];
    y[threadIdx.x] = hdr->y[threadIdx.x];
  }
  __syncthreads();
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= g.R) return;
  double2 u[KR];
#pragma unroll
  for (int a = 0; a < KR; ++a) {
    u[a] = make_double2(0.0, 0.0);
    if (a < s) {
      const int c = S[a];
      u[a] = (r == c) ? diag64[r] : St<T>::to_d(G[g_at(g, r, c)]);
    }
  }
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < KR; ++a)
    if (a < s) acc = cadd(acc, cmul(u[a], y[a]));
  double2* urow = U64 + (int64_t)r * KR;
#pragma unroll
  for (int a = 0; a < KR; ++a) urow[a] = u[a];
  if (bf16) {
    __bf16* arow = Abf + (int64_t)r * 2 * KP;
#pragma unroll
    for (int a0 = 0; a0 < KR; a0 += 8) {
      if (a0 < KP) {
        bf16x8v re, im;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          re[i] = (__bf16)(float)u[a0 + i].x;
          im[i] = (__bf16)(float)u[a0 + i].y;
        }
        *reinterpret_cast<bf16x8v*>(arow + a0) = re;
        *reinterpret_cast<bf16x8v*>(arow + KP + a0) = im;
      }
    }
  } else {
    float* arow = Af + (int64_t)r * 2 * KP;
#pragma unroll
    for (int a0 = 0; a0 < KR; a0 += 4) {
      if (a0 < KP) {
        const f32x4v re = {(float)u[a0].x, (float)u[a0 + 1].x, (float)u[a0 + 2].x, (float)u[a0 + 3].x};
        const f32x4v im = {(float)u[a0].y, (float)u[a0 + 1].y, (float)u[a0 + 2].y, (float)u[a0 + 3].y};
        *reinterpret_cast<f32x4v*>(arow + a0) = re;
        *reinterpret_cast<f32x4v*>(arow + KP + a0) = im;
      }
    }
  }
  E[r] = St<T>::from_d(cadd(St<T>::to_d(E[r]), acc));
}

// ------------------------------------------------------------------ RK3: columns (W = M G[S, :])
// One thread per column in 64-thread workgroups; M (FP64, KR x KR) is staged
// in LDS and read as a broadcast.  B operands per column [q][out][kappa]: out 0
// (real part of the product): [Re W ; -Im W], out 1 (imaginary part):
// [Im W ; Re W], written with 16-byte stores.  diag64 += diag(U W).
template <typename T>
__global__ __launch_bounds__(64) void k_rk_cols(Geo g, const RkHdr* __restrict__ hdr,
                                                const double2* __restrict__ M,
                                                const T* __restrict__ G,
                                                double2* __restrict__ diag64,
                                                const double2* __restrict__ U64,
                                                float* __restrict__ Bf, __bf16* __restrict__ Bbf,
                                                int bf16) {
  __shared__ double2 sM[KR * KR];
  __shared__ int S[KR];
  const int s = hdr->s;
  if (s == 0) return;
  const int KP = hdr->kp;
  for (int i = threadIdx.x; i < KR * KR; i += 64) sM[i] = M[i];
  if (threadIdx.x < KR) S[threadIdx.x] = hdr->S[threadIdx.x];
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (q >= g.ld) return;
  double2 gs[KR];
#pragma unroll
  for (int b = 0; b < KR; ++b) {
    gs[b] = make_double2(0.0, 0.0);
    if (b < s && q < g.N) {
      const int c = S[b];
      gs[b] = (q == c) ? diag64[c] : St<T>::to_d(G[g_at(g, c, q)]);
    }
  }
  double2 dsum = make_double2(0.0, 0.0);
  const int64_t base = q * 4 * KP;
#pragma unroll
  for (int a0 = 0; a0 < KR; a0 += 8) {
    if (a0 < KP) {
      double2 w[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        w[i] = make_double2(0.0, 0.0);
        if (a0 + i < s) {
#pragma unroll
          for (int b = 0; b < KR; ++b)
            if (b < s) w[i] = cadd(w[i], cmul(sM[(a0 + i) * KR + b], gs[b]));
          if (q < g.N) dsum = cadd(dsum, cmul(U64[q * KR + a0 + i], w[i]));
        }
      }
      if (bf16) {
        bf16x8v wr, wi, nwi;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          wr[i] = (__bf16)(float)w[i].x;
          wi[i] = (__bf16)(float)w[i].y;
          nwi[i] = (__bf16)(float)(-w[i].y);
        }
        *reinterpret_cast<bf16x8v*>(Bbf + base + a0) = wr;
        *reinterpret_cast<bf16x8v*>(Bbf + base + KP + a0) = nwi;
        *reinterpret_cast<bf16x8v*>(Bbf + base + 2 * KP + a0) = wi;
        *reinterpret_cast<bf16x8v*>(Bbf + base + 3 * KP + a0) = wr;
      } else {
#pragma unroll
        for (int j = 0; j < 8; j += 4) {
          const f32x4v wr = {(float)w[j].x, (float)w[j + 1].x, (float)w[j + 2].x, (float)w[j + 3].x};
          const f32x4v wi = {(float)w[j].y, (float)w[j + 1].y, (float)w[j + 2].y, (float)w[j + 3].y};
          const f32x4v nwi = {-wi[0], -wi[1], -wi[2], -wi[3]};
          *reinterpret_cast<f32x4v*>(Bf + base + a0 + j) = wr;
          *reinterpret_cast<f32x4v*>(Bf + base + KP + a0 + j) = nwi;
          *reinterpret_cast<f32x4v*>(Bf + base + 2 * KP + a0 + j) = wi;
          *reinterpret_cast<f32x4v*>(Bf + base + 3 * KP + a0 + j) = wr;
        }
      }
    }
  }
  if (q < g.N) diag64[q] = cadd(diag64[q], dsum);
}

// ------------------------------------------------------------------ RK4: MFMA update
// A workgroup of rows [r0, r0 + nr) and columns below c_end is left out when it
// lies wholly in design rows (r0 + nr <= skip_below = N) and strictly below the
// diagonal tiles (c_end <= r0, r0 a multiple of 64): with the design block's
// upper triangle kept alone (deferred mode, or state.lower_stale), those
// entries are never read.  skip_below = 0 updates every entry.
__device__ __forceinline__ bool rk_below_diagonal(int r0, int nr, int64_t c_end, int skip_below) {
  return skip_below > 0 && r0 + nr <= skip_below && c_end <= r0;
}


// Workgroup: 4 waves over a 64 x 64 complex tile per iteration (wave w: column
// tile w & 1, row tile w >> 1), RBLK row blocks of 64 rows per workgroup.  The
// A rows of the iteration are staged in LDS and shared by the two column waves;
// each wave keeps its B fragment in registers for the whole workgroup.
// 32x32 accumulator layout: element e of lane l is row 8*(e/4) + 4*(l/32) + e%4,
// column l%32.
constexpr int kRkRowBlocks = 8;

template <int KP, bool BF16>
__global__ __launch_bounds__(256) void k_rk_mfma(int R, int64_t ld, int skip_below,
                                                 const int32_t* __restrict__ gate_count,
                                                 const int32_t* __restrict__ gate_kp,
                                                 const float* __restrict__ Af,
                                                 const float* __restrict__ Bf,
                                                 const __bf16* __restrict__ Abf,
                                                 const __bf16* __restrict__ Bbf,
                                                 float2* __restrict__ G) {
  // gate_count: number of active terms (0 = nothing to do); gate_kp: the rank
  // padding chosen on the device (the instantiation that does not match exits)
  if (*gate_count == 0 || (gate_kp != nullptr && *gate_kp != KP)) return;
  constexpr int K2 = 2 * KP;
  constexpr int PADF = BF16 ? 4 : 1;   // LDS row padding (floats): 16-B rows for BF16, odd stride for FP32
  __shared__ __attribute__((aligned(16))) float sA[64 * (K2 + PADF)];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ncg = (int)(ld / 64);
  int cg, rg;
  ut_group(blockIdx.x, ncg, skip_below / (64 * kRkRowBlocks), 64 * kRkRowBlocks, 64, rg, cg);
  const int q = cg * 64 + (w & 1) * 32 + (lane & 31);
  const int h = lane >> 5;
  // B fragments for this lane's column
  constexpr int NB = BF16 ? K2 / 16 : KP;                 // MFMA instructions per output
  float bre[BF16 ? 1 : KP], bim[BF16 ? 1 : KP];
  bf16x8 bre8[BF16 ? NB : 1], bim8[BF16 ? NB : 1];
  if constexpr (BF16) {
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      bre8[t] = *reinterpret_cast<const bf16x8*>(Bbf + (int64_t)q * 2 * K2 + 16 * t + 8 * h);
      bim8[t] = *reinterpret_cast<const bf16x8*>(Bbf + (int64_t)q * 2 * K2 + K2 + 16 * t + 8 * h);
    }
  } else {
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      bre[t] = Bf[(int64_t)q * 2 * K2 + h * KP + t];
      bim[t] = Bf[(int64_t)q * 2 * K2 + K2 + h * KP + t];
    }
  }
  for (int rb = 0; rb < kRkRowBlocks; ++rb) {
    const int r0 = (rg * kRkRowBlocks + rb) * 64;
    if (r0 >= R) break;
    __syncthreads();
    // stage A rows [r0, r0 + 64) in LDS (FP32 or BF16 bits, K2 values per row)
    if constexpr (BF16) {
      constexpr int per_row = K2 / 8;                     // 16-byte chunks per row
      for (int c = threadIdx.x; c < 64 * per_row; c += 256) {
        const int rr = c / per_row, cc = c - (c / per_row) * per_row;
        const int r = r0 + rr;
        f32x4v v = {0.f, 0.f, 0.f, 0.f};
        if (r < R) v = *reinterpret_cast<const f32x4v*>(Abf + (int64_t)r * K2 + 8 * cc);
        *reinterpret_cast<f32x4v*>(&sA[rr * (K2 + PADF) + 4 * cc]) = v;
      }
    } else {
      for (int c = threadIdx.x; c < 64 * K2; c += 256) {
        const int rr = c / K2, cc = c - (c / K2) * K2;
        const int r = r0 + rr;
        sA[rr * (K2 + PADF) + cc] = (r < R) ? Af[(int64_t)r * K2 + cc] : 0.f;
      }
    }
    __syncthreads();
    const int rt = r0 + (w >> 1) * 32;
    // load the G tile into the accumulators
    f32x16 accr, acci;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int r = rt + 8 * (e >> 2) + 4 * h + (e & 3);
      float2 gv = make_float2(0.f, 0.f);
      if (r < R) gv = G[(int64_t)r * ld + q];
      accr[e] = gv.x;
      acci[e] = gv.y;
    }
    const float* arow = &sA[((w >> 1) * 32 + (lane & 31)) * (K2 + PADF)];
    if constexpr (BF16) {
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const bf16x8 a8 = *reinterpret_cast<const bf16x8*>(
            reinterpret_cast<const __bf16*>(arow) + 16 * t + 8 * h);
        accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, bre8[t], accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, bim8[t], acci, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int t = 0; t < KP; ++t) {
        const float a = arow[h * KP + t];
        accr = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bre[t], accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bim[t], acci, 0, 0, 0);
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int r = rt + 8 * (e >> 2) + 4 * h + (e & 3);
      if (r < R) G[(int64_t)r * ld + q] = make_float2(accr[e], acci[e]);
    }
  }
}

// ------------------------------------------------------------------ RK4': streaming MFMA update
// Workgroup: 4 waves side by side over 128 columns (wave w: columns
// cg * 128 + 32 w ..), RB blocks of 32 rows.  The workgroup's A rows (RB x 32
// rows x 2 KP) are staged in LDS once; B fragments stay in registers.  In each
// row block a wave first requests its G entries, then forms the product from
// zero accumulators (no matrix instruction waits for G), then adds G and
// stores, so the G loads are in flight during the products.
//   LDSEPI = false: G in the accumulator layout (8 bytes per lane, 256-byte row
//     segments per half-wave), no barrier in the row loop;
//   LDSEPI = true: the 32 x 128 product goes through LDS and G streams in
//     16-byte pieces (1 KB row segments per wave), two barriers per row block.
// G is read and written with non-temporal (streaming) loads and stores.
// The launch bound keeps the FP32 rank-16 forms with one row tile and four row
// blocks within 128 registers (about 120 needed): three to four waves per SIMD,
// as LDS allows, and more loads of G in flight than at two.
template <int KP, bool BF16, int RB, bool LDSEPI, int TM = 1>
__global__ __launch_bounds__(256, (!BF16 && TM == 1 && KP == 16 && RB <= 4) ? 3 : 1) void k_rk_stream(int R, int64_t ld, int skip_below,
                                                   const int32_t* __restrict__ gate_count,
                                                   const int32_t* __restrict__ gate_kp,
                                                   const float* __restrict__ Af,
                                                   const float* __restrict__ Bf,
                                                   const __bf16* __restrict__ Abf,
                                                   const __bf16* __restrict__ Bbf,
                                                   float2* __restrict__ G) {
  if (*gate_count == 0 || *gate_kp != KP) return;
  constexpr int K2 = 2 * KP;
  // LDS row width (floats): odd for FP32 (conflict-free column reads), 16-byte
  // rows plus 16 bytes of padding for BF16
  constexpr int AW = BF16 ? K2 / 2 + 4 : K2 + 1;
  constexpr int PW = 130;                           // product tile row width (float2)
  static_assert(!LDSEPI || TM == 1, "the LDS epilogue takes one row tile per wave");
  constexpr int BR = 32 * TM;                       // rows per block
  __shared__ __attribute__((aligned(16))) float sA[RB * BR * AW];
  __shared__ __attribute__((aligned(16))) float2 sP[LDSEPI ? 32 * PW : 2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, h = lane >> 5;
  const int ncg = (int)((ld + 127) / 128);
  int cg, rg;
  ut_group(blockIdx.x, ncg, skip_below / (RB * BR), RB * BR, 128, rg, cg);
  const int64_t c0 = (int64_t)cg * 128;
  const int rbase = rg * RB * BR;
  const int64_t q = c0 + 32 * w + (lane & 31);
  const bool qok = q < ld;
  // A rows of the workgroup
  if constexpr (BF16) {
    constexpr int per_row = K2 / 8;                   // 16-byte chunks per row
    for (int c = threadIdx.x; c < RB * BR * per_row; c += 256) {
      const int rr = c / per_row, cc = c - (c / per_row) * per_row;
      const int r = rbase + rr;
      f32x4v v = {0.f, 0.f, 0.f, 0.f};
      if (r < R) v = *reinterpret_cast<const f32x4v*>(Abf + (int64_t)r * K2 + 8 * cc);
      *reinterpret_cast<f32x4v*>(&sA[rr * AW + 4 * cc]) = v;
    }
  } else {
    for (int c = threadIdx.x; c < RB * BR * K2; c += 256) {
      const int rr = c / K2, cc = c - (c / K2) * K2;
      const int r = rbase + rr;
      sA[rr * AW + cc] = (r < R) ? Af[(int64_t)r * K2 + cc] : 0.f;
    }
  }
  // B fragments of this lane's column
  constexpr int NB = BF16 ? K2 / 16 : KP;
  float bre[BF16 ? 1 : KP], bim[BF16 ? 1 : KP];
  bf16x8 bre8[BF16 ? NB : 1], bim8[BF16 ? NB : 1];
  if constexpr (BF16) {
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      bre8[t] = bf16x8{};
      bim8[t] = bf16x8{};
      if (qok) {
        bre8[t] = *reinterpret_cast<const bf16x8*>(Bbf + q * 2 * K2 + 16 * t + 8 * h);
        bim8[t] = *reinterpret_cast<const bf16x8*>(Bbf + q * 2 * K2 + K2 + 16 * t + 8 * h);
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < KP; t += 4) {
      f32x4v vr = {0.f, 0.f, 0.f, 0.f}, vi = {0.f, 0.f, 0.f, 0.f};
      if (qok) {
        vr = *reinterpret_cast<const f32x4v*>(Bf + q * 2 * K2 + h * KP + t);
        vi = *reinterpret_cast<const f32x4v*>(Bf + q * 2 * K2 + K2 + h * KP + t);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        bre[t + i] = vr[i];
        bim[t + i] = vi[i];
      }
    }
  }
  __syncthreads();
  // the epilogue layout of the LDS form: thread t takes rows (t >> 6) + 4 i of
  // the block and the two columns c0 + 2 (t & 63), + 1
  const int64_t qc = c0 + 2 * (threadIdx.x & 63);
  const bool cok = qc < ld;                           // ld is a multiple of 64
  for (int rb = 0; rb < RB; ++rb) {
    const int r0 = rbase + rb * BR;
    if (r0 >= R) break;                               // uniform across the workgroup
    f32x2v gacc[LDSEPI ? 1 : 16 * TM];
    f32x4v g16[LDSEPI ? 8 : 1];
    if constexpr (LDSEPI) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = r0 + (threadIdx.x >> 6) + 4 * i;
        g16[i] = f32x4v{0.f, 0.f, 0.f, 0.f};
        if (cok && r < R)
          g16[i] = __builtin_nontemporal_load(reinterpret_cast<const f32x4v*>(G + (int64_t)r * ld + qc));
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16 * TM; ++e) {
        const int r = r0 + 32 * (e >> 4) + 8 * ((e & 15) >> 2) + 4 * h + (e & 3);
        gacc[e] = f32x2v{0.f, 0.f};
        if (qok && r < R)
          gacc[e] = __builtin_nontemporal_load(reinterpret_cast<const f32x2v*>(G + (int64_t)r * ld + q));
      }
    }
    // keep the G requests ahead of the products
    __builtin_amdgcn_sched_barrier(0);
    f32x16 accr[TM], acci[TM];
#pragma unroll
    for (int tm = 0; tm < TM; ++tm) {
      accr[tm] = f32x16{};
      acci[tm] = f32x16{};
      const float* arow = &sA[(rb * BR + 32 * tm + (lane & 31)) * AW];
      if constexpr (BF16) {
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const bf16x8 a8 = *reinterpret_cast<const bf16x8*>(
              reinterpret_cast<const __bf16*>(arow) + 16 * t + 8 * h);
          accr[tm] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, bre8[t], accr[tm], 0, 0, 0);
          acci[tm] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, bim8[t], acci[tm], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int t = 0; t < KP; ++t) {
          const float av = arow[h * KP + t];
          accr[tm] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bre[t], accr[tm], 0, 0, 0);
          acci[tm] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bim[t], acci[tm], 0, 0, 0);
        }
      }
    }
    if constexpr (LDSEPI) {
      __syncthreads();                                // the previous block's product is read
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int rr = 8 * (e >> 2) + 4 * h + (e & 3);
        sP[rr * PW + 32 * w + (lane & 31)] = make_float2(accr[0][e], acci[0][e]);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int rl = (threadIdx.x >> 6) + 4 * i;
        const int r = r0 + rl;
        if (cok && r < R) {
          const f32x4v pv = *reinterpret_cast<const f32x4v*>(&sP[rl * PW + 2 * (threadIdx.x & 63)]);
          const f32x4v o = g16[i] + pv;
          __builtin_nontemporal_store(o, reinterpret_cast<f32x4v*>(G + (int64_t)r * ld + qc));
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16 * TM; ++e) {
        const int r = r0 + 32 * (e >> 4) + 8 * ((e & 15) >> 2) + 4 * h + (e & 3);
        if (qok && r < R) {
          const f32x2v o = {gacc[e][0] + accr[e >> 4][e & 15], gacc[e][1] + acci[e >> 4][e & 15]};
          __builtin_nontemporal_store(o, reinterpret_cast<f32x2v*>(G + (int64_t)r * ld + q));
        }
      }
    }
  }
}

// Update variants (autotuner): the 64 x 64 form that accumulates the products
// onto G (k_rk_mfma) and the streaming forms above with 4 or 8 row blocks per
// workgroup.  The streaming forms sum the products from zero in the same order
// and add G once, so they agree with each other bit for bit; against the
// accumulating form they differ by FP32 rounding.
static const char* const kRkNames[] = {"acc64",     "pre128_r4",   "pre128_r8",  "lds128_r4",
                                       "lds128_r8", "pre128t2_r2", "pre128t2_r4"};
constexpr int kRkCount = (int)(sizeof(kRkNames) / sizeof(kRkNames[0]));
static std::atomic<int> g_rk_sel{0};
int rk_variant_count() { return kRkCount; }
const char* rk_variant_name(int i) { return i >= 0 && i < kRkCount ? kRkNames[i] : nullptr; }
int rk_set_variant(int i) {
  if (i < 0 || i >= kRkCount) return GFO_EINVAL;
  g_rk_sel.store(i);
  return GFO_OK;
}
int rk_get_variant() { return g_rk_sel.load(); }

template <bool BF16, int RB, bool LDSEPI, int TM = 1>
static void launch_rk_stream(const Geo& g, RkHdr* hdr, const float* Af, const float* Bf,
                             const __bf16* Abf, const __bf16* Bbf, float2* G, hipStream_t s) {
  const int ncg = (int)((g.ld + 127) / 128);
  const int H = 32 * TM * RB, nrg = (g.R + H - 1) / H;
  const int skip = g.upper ? g.N : 0;
  const dim3 grid((unsigned)ut_group_count(nrg, ncg, skip / H, H, 128));
  hipLaunchKernelGGL((k_rk_stream<16, BF16, RB, LDSEPI, TM>), grid, dim3(256), 0, s, g.R, g.ld, skip,
                     &hdr->s, &hdr->kp, Af, Bf, Abf, Bbf, G);
  hipLaunchKernelGGL((k_rk_stream<32, BF16, RB, LDSEPI, TM>), grid, dim3(256), 0, s, g.R, g.ld, skip,
                     &hdr->s, &hdr->kp, Af, Bf, Abf, Bbf, G);
}

hipError_t launch_rank_k(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* picks, int k,
                         int precision, hipStream_t s) {
  if (g.dtype != GFO_C64) return note_hip(hipErrorInvalidValue);
  char* w = (char*)st->work;
  RkHdr* hdr = (RkHdr*)(w + L.rk_S);
  double2* M = (double2*)(w + L.rk_M);
  double2* U64 = (double2*)(w + L.rk_U64);
  float* Af = (float*)(w + L.rk_A);
  float* Bf = (float*)(w + L.rk_B);
  __bf16* Abf = (__bf16*)(w + L.rk_Abf);
  __bf16* Bbf = (__bf16*)(w + L.rk_Bbf);
  const int bf = precision == GFO_BF16 ? 1 : 0;
  float2* G = (float2*)st->G;
  hipLaunchKernelGGL(k_rk_prepare<float2>, dim3(1), dim3(256), 0, s, g, picks, k,
                     (const float2*)G, (const float2*)st->E, (const double2*)st->diag64,
                     st->eps_idx, st->flips, st->flip_cap, st->n_flips, st->status, hdr, M);
  hipLaunchKernelGGL(k_rk_rows<float2>, dim3((g.R + 63) / 64), dim3(64), 0, s, g,
                     (const RkHdr*)hdr, (const float2*)G, (const double2*)st->diag64,
                     (float2*)st->E, U64, Af, Abf, bf);
  hipLaunchKernelGGL(k_rk_cols<float2>, dim3((unsigned)((g.ld + 63) / 64)), dim3(64), 0, s, g,
                     (const RkHdr*)hdr, (const double2*)M, (const float2*)G,
                     (double2*)st->diag64, (const double2*)U64, Bf, Bbf, bf);
  hipEvent_t before, after;
  k1_take_timing(&before, &after);
  if (hipError_t er = record_event(before, s)) return note_hip(er);
  // the rank padding (16 or 32) is decided on the device; both instantiations are
  // launched and the one that does not match exits at once
  const float* cAf = Af;
  const float* cBf = Bf;
  const __bf16* cAbf = Abf;
  const __bf16* cBbf = Bbf;
  switch (rk_get_variant()) {
    case 1:
      if (bf) launch_rk_stream<true, 4, false>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      else launch_rk_stream<false, 4, false>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      break;
    case 2:
      if (bf) launch_rk_stream<true, 8, false>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      else launch_rk_stream<false, 8, false>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      break;
    case 3:
      if (bf) launch_rk_stream<true, 4, true>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      else launch_rk_stream<false, 4, true>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      break;
    case 4:
      if (bf) launch_rk_stream<true, 8, true>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      else launch_rk_stream<false, 8, true>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      break;
    case 5:
      if (bf) launch_rk_stream<true, 2, false, 2>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      else launch_rk_stream<false, 2, false, 2>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      break;
    case 6:
      if (bf) launch_rk_stream<true, 4, false, 2>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      else launch_rk_stream<false, 4, false, 2>(g, hdr, cAf, cBf, cAbf, cBbf, G, s);
      break;
    default: {
      const int ncg = (int)(g.ld / 64);
      const int H = 64 * kRkRowBlocks, nrg = (g.R + H - 1) / H;
      const int skip = g.upper ? g.N : 0;
      const dim3 grid((unsigned)ut_group_count(nrg, ncg, skip / H, H, 64));
      if (bf) {
        hipLaunchKernelGGL((k_rk_mfma<16, true>), grid, dim3(256), 0, s, g.R, g.ld, skip, &hdr->s,
                           &hdr->kp, cAf, cBf, cAbf, cBbf, G);
        hipLaunchKernelGGL((k_rk_mfma<32, true>), grid, dim3(256), 0, s, g.R, g.ld, skip, &hdr->s,
                           &hdr->kp, cAf, cBf, cAbf, cBbf, G);
      } else {
        hipLaunchKernelGGL((k_rk_mfma<16, false>), grid, dim3(256), 0, s, g.R, g.ld, skip, &hdr->s,
                           &hdr->kp, cAf, cBf, cAbf, cBbf, G);
        hipLaunchKernelGGL((k_rk_mfma<32, false>), grid, dim3(256), 0, s, g.R, g.ld, skip, &hdr->s,
                           &hdr->kp, cAf, cBf, cAbf, cBbf, G);
      }
      break;
    }
  }
  if (hipError_t er = record_event(after, s)) return note_hip(er);
  return note_hip(hipGetLastError());
}

}  // namespace gfo
