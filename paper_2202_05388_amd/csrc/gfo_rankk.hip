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

namespace gfo {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
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
// U64 (R x KR, FP64), A operand row-major [r][kappa], kappa < KP: Re U, kappa >= KP: Im U,
// in FP32 (Af) and BF16 (Abf); E += U y.
template <typename T>
__global__ void k_rk_rows(Geo g, const RkHdr* __restrict__ hdr, const T* __restrict__ G,
                          const double2* __restrict__ diag64, T* __restrict__ E,
                          double2* __restrict__ U64, float* __restrict__ Af,
                          __bf16* __restrict__ Abf, int bf16) {
  const int s = hdr->s;
  if (s == 0) return;
  const int KP = hdr->kp;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.R) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int a = 0; a < KP; ++a) {
    double2 u = make_double2(0.0, 0.0);
    if (a < s) {
      const int c = hdr->S[a];
      u = (r == c) ? diag64[r] : St<T>::to_d(G[g_at(g, r, c)]);
      acc = cadd(acc, cmul(u, hdr->y[a]));
    }
    U64[(int64_t)r * KR + a] = u;
    if (bf16) {
      Abf[(int64_t)r * 2 * KP + a] = (__bf16)(float)u.x;
      Abf[(int64_t)r * 2 * KP + KP + a] = (__bf16)(float)u.y;
    } else {
      Af[(int64_t)r * 2 * KP + a] = (float)u.x;
      Af[(int64_t)r * 2 * KP + KP + a] = (float)u.y;
    }
  }
  E[r] = St<T>::from_d(cadd(St<T>::to_d(E[r]), acc));
}

// ------------------------------------------------------------------ RK3: columns (W = M G[S, :])
// B operands column-major [q][out][kappa]: out 0 (real part of the product):
// [Re W ; -Im W], out 1 (imaginary part): [Im W ; Re W].  diag64 += diag(U W).
template <typename T>
__global__ void k_rk_cols(Geo g, const RkHdr* __restrict__ hdr, const double2* __restrict__ M,
                          const T* __restrict__ G, double2* __restrict__ diag64,
                          const double2* __restrict__ U64, float* __restrict__ Bf,
                          __bf16* __restrict__ Bbf, int bf16) {
  const int s = hdr->s;
  if (s == 0) return;
  const int KP = hdr->kp;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.ld) return;
  double2 gs[KR];
#pragma unroll
  for (int b = 0; b < KR; ++b) {
    gs[b] = make_double2(0.0, 0.0);
    if (b < s && q < g.N) {
      const int c = hdr->S[b];
      gs[b] = (q == c) ? diag64[c] : St<T>::to_d(G[g_at(g, c, q)]);
    }
  }
  double2 dsum = make_double2(0.0, 0.0);
  for (int a = 0; a < KP; ++a) {
    double2 w = make_double2(0.0, 0.0);
    if (a < s) {
#pragma unroll
      for (int b = 0; b < KR; ++b)
        if (b < s) w = cadd(w, cmul(M[a * KR + b], gs[b]));
      if (q < g.N) dsum = cadd(dsum, cmul(U64[q * KR + a], w));
    }
    const int64_t base = q * 4 * KP;
    if (bf16) {
      Bbf[base + a] = (__bf16)(float)w.x;
      Bbf[base + KP + a] = (__bf16)(float)(-w.y);
      Bbf[base + 2 * KP + a] = (__bf16)(float)w.y;
      Bbf[base + 3 * KP + a] = (__bf16)(float)w.x;
    } else {
      Bf[base + a] = (float)w.x;
      Bf[base + KP + a] = (float)(-w.y);
      Bf[base + 2 * KP + a] = (float)w.y;
      Bf[base + 3 * KP + a] = (float)w.x;
    }
  }
  if (q < g.N) diag64[q] = cadd(diag64[q], dsum);
}

// ------------------------------------------------------------------ RK4: MFMA update
// Workgroup: 4 waves over a 64 x 64 complex tile per iteration (wave w: column
// tile w & 1, row tile w >> 1), RBLK row blocks of 64 rows per workgroup.  The
// A rows of the iteration are staged in LDS and shared by the two column waves;
// each wave keeps its B fragment in registers for the whole workgroup.
// 32x32 accumulator layout: element e of lane l is row 8*(e/4) + 4*(l/32) + e%4,
// column l%32.
constexpr int kRkRowBlocks = 8;

template <int KP, bool BF16>
__global__ __launch_bounds__(256) void k_rk_mfma(int R, int64_t ld,
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
  const int cg = blockIdx.x % ncg, rg = blockIdx.x / ncg;
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

hipError_t launch_rank_k(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* picks, int k,
                         int precision, hipStream_t s) {
  if (g.dtype != GFO_C64) return hipErrorInvalidValue;
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
  hipLaunchKernelGGL(k_rk_rows<float2>, dim3((g.R + 255) / 256), dim3(256), 0, s, g,
                     (const RkHdr*)hdr, (const float2*)G, (const double2*)st->diag64,
                     (float2*)st->E, U64, Af, Abf, bf);
  hipLaunchKernelGGL(k_rk_cols<float2>, dim3((unsigned)((g.ld + 255) / 256)), dim3(256), 0, s, g,
                     (const RkHdr*)hdr, (const double2*)M, (const float2*)G,
                     (double2*)st->diag64, (const double2*)U64, Bf, Bbf, bf);
  const int ncg = (int)(g.ld / 64);
  const int nrg = (g.R + 64 * kRkRowBlocks - 1) / (64 * kRkRowBlocks);
  const dim3 grid((unsigned)(ncg * nrg));
  hipEvent_t before, after;
  k1_take_timing(&before, &after);
  if (before && hipEventRecord(before, s) != hipSuccess) return hipErrorUnknown;
  // the rank padding (16 or 32) is decided on the device; both instantiations are
  // launched and the one that does not match exits at once
  if (bf) {
    hipLaunchKernelGGL((k_rk_mfma<16, true>), grid, dim3(256), 0, s, g.R, g.ld, &hdr->s, &hdr->kp,
                       (const float*)Af, (const float*)Bf, (const __bf16*)Abf, (const __bf16*)Bbf, G);
    hipLaunchKernelGGL((k_rk_mfma<32, true>), grid, dim3(256), 0, s, g.R, g.ld, &hdr->s, &hdr->kp,
                       (const float*)Af, (const float*)Bf, (const __bf16*)Abf, (const __bf16*)Bbf, G);
  } else {
    hipLaunchKernelGGL((k_rk_mfma<16, false>), grid, dim3(256), 0, s, g.R, g.ld, &hdr->s, &hdr->kp,
                       (const float*)Af, (const float*)Bf, (const __bf16*)Abf, (const __bf16*)Bbf, G);
    hipLaunchKernelGGL((k_rk_mfma<32, false>), grid, dim3(256), 0, s, g.R, g.ld, &hdr->s, &hdr->kp,
                       (const float*)Af, (const float*)Bf, (const __bf16*)Abf, (const __bf16*)Bbf, G);
  }
  if (after && hipEventRecord(after, s) != hipSuccess) return hipErrorUnknown;
  return hipGetLastError();
}

}  // namespace gfo
