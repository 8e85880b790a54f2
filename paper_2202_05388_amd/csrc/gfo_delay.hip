// Deferred rank-1 updates.  Eq. form10 applied move by move gives
//   G_t = G_base + sum_{s < t} cu_s v_s^T,   cu_s = c_s G_s[:, j_s],  v_s = G_s[j_s, :],
// so the design block can be brought up to date later, in one rank-r product,
// while everything the scores read (E, diag64, the monitor rows) is updated at
// once.  Column j and row j of the current matrix are the base entries plus the
// pending terms.
#include "gfo_internal.hpp"

#include <atomic>

namespace gfo {

// Pending terms are stored twice: element-major, CU[r * D + s] and V[q * D + s]
// (D = GFO_MAX_DELAY; the terms of one element are contiguous, which the
// per-step gathers read), and slot-major, CUs[s * R + r] and Vs[s * ld + q]
// (consecutive elements of one term are contiguous, which the flush reads
// coalesced across lanes).
constexpr int D = GFO_MAX_DELAY;

// The move's scalars, computed by every thread from values no thread of this
// launch writes (pick, eps_idx[j], diag64[j], E[j], the term count).
template <typename T>
__device__ __forceinline__ Snap deferred_snapshot(const Geo& g, const gfo_pick* __restrict__ pick,
                                                  const T* __restrict__ E,
                                                  const double2* __restrict__ diag64,
                                                  const uint8_t* __restrict__ eps_idx,
                                                  const int32_t* __restrict__ count) {
  Snap s = {};
  s.j = -1;
  const int j = pick->pixel, e = pick->eps_idx;
  if (j >= 0 && j < g.N && e >= 0 && e < g.n_eps && e != (int)eps_idx[j]) {
    const double a = g.k0sq * (g.eps[e] - g.eps[eps_idx[j]]);
    const double2 d = diag64[j];
    const double2 den = make_double2(1.0 - a * d.x, -a * d.y);
    if (cabs2(den) < 1e-24) {
      s.pad1 = 1;                           // singular: refused, flagged by the next kernel
    } else {
      s.j = j;
      s.e_new = e;
      s.alpha = a;
      s.c = rdiv(a, den);
      s.Ej = St<T>::to_d(E[j]);
      s.dj = d;
      s.slot = *count;
    }
  }
  return s;
}

// Threads [0, R): u_r = G_t[r, j] (base + pending for design rows; monitor rows
// are current); cu_r = c u_r is stored as term `slot` (both layouts) and in `cu`.
// Threads [R, R + ld): v_q = G_t[j, q] (q < N, 0 beyond), stored likewise and in
// `v`.  Workgroup 0 publishes the snapshot for the next kernel.  This kernel
// writes nothing that it reads.
template <typename T>
__global__ void k_gather_dl(Geo g, const gfo_pick* __restrict__ pick, const T* __restrict__ G,
                            const T* __restrict__ E, const double2* __restrict__ diag64,
                            const uint8_t* __restrict__ eps_idx, const int32_t* __restrict__ count,
                            Snap* __restrict__ snap_out, T* __restrict__ CU, T* __restrict__ V,
                            T* __restrict__ CUs, T* __restrict__ Vs, T* __restrict__ cu_out,
                            T* __restrict__ v_out) {
  const Snap sn = deferred_snapshot<T>(g, pick, E, diag64, eps_idx, count);
  if (blockIdx.x == 0 && threadIdx.x == 0) *snap_out = sn;
  const int j = sn.j;
  if (j < 0) return;
  const int slot = sn.slot;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < g.R) {
    const int64_t i = t;
    double2 u;
    if (i == j) {
      u = sn.dj;
    } else {
      u = St<T>::to_d(G[i * g.ld + j]);
      if (i < g.N) {
        const T* __restrict__ cr = CU + i * D;
        const T* __restrict__ vj = V + (int64_t)j * D;
#pragma unroll 8
        for (int s = 0; s < slot; ++s) u = cadd(u, cmul(St<T>::to_d(cr[s]), St<T>::to_d(vj[s])));
      }
    }
    const T cu = St<T>::from_d(cmul(sn.c, u));
    CU[i * D + slot] = cu;
    CUs[(int64_t)slot * g.R + i] = cu;
    cu_out[i] = cu;
  } else if (t < g.R + g.ld) {
    const int64_t q = t - g.R;
    double2 v = make_double2(0.0, 0.0);
    if (q < g.N) {
      if (q == j) {
        v = sn.dj;
      } else {
        v = St<T>::to_d(G[(int64_t)j * g.ld + q]);
        const T* __restrict__ cj = CU + (int64_t)j * D;
        const T* __restrict__ vq = V + q * D;
#pragma unroll 8
        for (int s = 0; s < slot; ++s) v = cadd(v, cmul(St<T>::to_d(cj[s]), St<T>::to_d(vq[s])));
      }
    }
    const T vv = St<T>::from_d(v);
    V[q * D + slot] = vv;
    Vs[(int64_t)slot * g.ld + q] = vv;
    v_out[q] = vv;
  }
}

// Applies the move's O(R) and O(N) parts: E_r += cu_r E_j for every row, the
// monitor rows G[N+m, q] += cu[N+m] v[q], diag64[q] += cu[q] v[q] (q != j),
// diag64[j] = d_j / (1 - alpha d_j); then records the move (eps_idx, history,
// move counter, term count).  Grid x covers max(R, ld); y walks the monitors.
template <typename T>
__global__ void k_mon_dl(Geo g, const Snap* __restrict__ snap, const T* __restrict__ cu,
                         const T* __restrict__ v, T* __restrict__ G, T* __restrict__ E,
                         double2* __restrict__ diag64, uint8_t* __restrict__ eps_idx,
                         int32_t* __restrict__ flips, int flip_cap, int32_t* __restrict__ n_flips,
                         int32_t* __restrict__ status, int32_t* __restrict__ count) {
  const int j = snap->j;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < 0) {
    if (q == 0 && blockIdx.y == 0 && snap->pad1) atomicOr(status, GFO_STATUS_SINGULAR);
    return;
  }
  if (blockIdx.y == 0) {
    if (q < g.R) E[q] = St<T>::from_d(cadd(St<T>::to_d(E[q]), cmul(St<T>::to_d(cu[q]), snap->Ej)));
    if (q < g.N) {
      if (q == j) {
        const double2 d = snap->dj;
        diag64[j] = cmul(d, rdiv(1.0, make_double2(1.0 - snap->alpha * d.x, -snap->alpha * d.y)));
      } else {
        diag64[q] = cadd(diag64[q], cmul(St<T>::to_d(cu[q]), St<T>::to_d(v[q])));
      }
    }
    if (q == 0) {
      eps_idx[j] = (uint8_t)snap->e_new;
      const int n = *n_flips;
      if (n < flip_cap) {
        flips[2 * n] = j;
        flips[2 * n + 1] = snap->e_new;
      } else {
        atomicOr(status, GFO_STATUS_HISTORY_FULL);
      }
      *n_flips = n + 1;
      *count = snap->slot + 1;
    }
  }
  if (q >= g.ld) return;
  const double2 vq = St<T>::to_d(v[q]);
  for (int m = blockIdx.y; m < g.nmon; m += gridDim.y) {
    const int64_t r = g.N + m;
    T* p = G + r * g.ld + q;
    *p = St<T>::from_d(cadd(St<T>::to_d(*p), cmul(St<T>::to_d(cu[r]), vq)));
  }
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// Fourth word of a raw buffer resource on gfx9-family chips (32-bit data format;
// reads past the range return zero).
constexpr int kBufferDword3 = 0x00020000;

// FP32 flush for complex64 storage: G[m, n] += sum_{s < count} CU[s][m] V[s][n]
// for design rows m < N and all ld columns, as complex FP32 on the matrix cores
// (v_mfma_f32_32x32x2_f32; re += Ar Br - Ai Bi, im += Ar Bi + Ai Br).  The G tile
// is loaded into the accumulators, so G is read and written once.  Workgroup of
// 4 waves = 64 x 64 outputs, each wave 32 x 32.  Lane layout of the instruction:
// A(i, k): i = lane % 32, k = lane / 32; B(k, j): j = lane % 32, k = lane / 32;
// accumulator element e: row 8*(e/4) + 4*(lane/32) + e%4, column lane % 32.
__global__ __launch_bounds__(256) void k_flush_c64(int M, int R, int64_t ld,
                                                   const int32_t* __restrict__ count,
                                                   const float2* __restrict__ CU,
                                                   const float2* __restrict__ V,
                                                   float2* __restrict__ G) {
  const int K = *count;
  if (K == 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int n = blockIdx.x * 64 + (w & 1) * 32 + (lane & 31);
  const int h = lane >> 5;
  f32x16 accr, acci;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = m0 + 8 * (e >> 2) + 4 * h + (e & 3);
    const float2 gv = row < M ? G[(int64_t)row * ld + n] : make_float2(0.f, 0.f);
    accr[e] = gv.x;
    acci[e] = gv.y;
  }
  const int am = m0 + (lane & 31);
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 2) {
    const int kk = k0 + h;
    float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
    if (kk < K) {
      if (am < M) a = CU[(int64_t)kk * R + am];
      b = V[(int64_t)kk * ld + n];
    }
    accr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, accr, 0, 0, 0);
    accr = __builtin_amdgcn_mfma_f32_32x32x2f32(-a.y, b.y, accr, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, acci, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, acci, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = m0 + 8 * (e >> 2) + 4 * h + (e & 3);
    if (row < M) G[(int64_t)row * ld + n] = make_float2(accr[e], acci[e]);
  }
}

// Same product with a 64 x 64 output tile per wave (2 x 2 instruction tiles) and
// 128 x 128 per workgroup, so each operand load feeds 8 instructions instead of 4.
// Workgroups are numbered XCD-aware: consecutive workgroup ids go to different
// XCDs (round robin), so id b is given to XCD b % 8, and each XCD walks its own
// band of row blocks; the A rows of a band then stay in that XCD's L2.
__global__ __launch_bounds__(256) void k_flush_c64_w64(int M, int R, int64_t ld, int nbx, int nby,
                                                       const int32_t* __restrict__ count,
                                                       const float2* __restrict__ CU,
                                                       const float2* __restrict__ V,
                                                       float2* __restrict__ G) {
  const int K = *count;
  if (K == 0) return;
  // XCD-aware tile order
  const int nxcd = 8;
  const int b = blockIdx.x;
  const int xcd = b % nxcd, local = b / nxcd;
  const int per = (nbx * nby + nxcd - 1) / nxcd;          // workgroups per XCD
  const int t = xcd * per + local;                        // position in row-major tile order
  if (t >= nbx * nby) return;
  const int by = t / nbx, bx = t - (t / nbx) * nbx;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = by * 128 + (w >> 1) * 64;
  const int n0 = bx * 128 + (w & 1) * 64;
  const int h = lane >> 5, l32 = lane & 31;
  f32x16 accr[2][2], acci[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const int n = n0 + 32 * tj + l32;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = m0 + 32 * ti + 8 * (e >> 2) + 4 * h + (e & 3);
        const float2 gv = (row < M && n < ld) ? G[(int64_t)row * ld + n] : make_float2(0.f, 0.f);
        accr[ti][tj][e] = gv.x;
        acci[ti][tj][e] = gv.y;
      }
    }
  for (int k0 = 0; k0 < K; k0 += 2) {
    const int kk = k0 + h;
    float2 a[2], bb[2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
      const int am = m0 + 32 * ti + l32;
      a[ti] = (kk < K && am < M) ? CU[(int64_t)kk * R + am] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const int n = n0 + 32 * tj + l32;
      bb[tj] = (kk < K && n < ld) ? V[(int64_t)kk * ld + n] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        accr[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ti].x, bb[tj].x, accr[ti][tj], 0, 0, 0);
        accr[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[ti].y, bb[tj].y, accr[ti][tj], 0, 0, 0);
        acci[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ti].x, bb[tj].y, acci[ti][tj], 0, 0, 0);
        acci[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ti].y, bb[tj].x, acci[ti][tj], 0, 0, 0);
      }
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const int n = n0 + 32 * tj + l32;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = m0 + 32 * ti + 8 * (e >> 2) + 4 * h + (e & 3);
        if (row < M && n < ld) G[(int64_t)row * ld + n] = make_float2(accr[ti][tj][e], acci[ti][tj][e]);
      }
    }
}

// Variants with TM row tiles of 32 per wave (a 32*TM x 32 output tile; the TM
// tiles share each B value) and 64*TM x 64 per workgroup.  The accumulators of
// different row tiles are independent, so consecutive matrix instructions do not
// wait on each other's results.  THREE_MULT uses three real products per complex
// product (Gauss): with P = sum Ar Br, Q = sum Ai Bi, S = sum (Ar + Ai)(Br + Bi),
// re = Gr + P - Q and im = Gi + S - P - Q; the accumulators start at X = Gr,
// Y = 0, Z = Gr + Gi, so that re = X - Y and im = Z - X - Y.  This removes a
// quarter of the matrix work; its rounding differs from the four-product form
// by a few units of FP32 in the last place relative to |G| + |CU||V|.
template <int TM, bool THREE_MULT>
__global__ __launch_bounds__(256) void k_flush_c64_tm(int M, int R, int64_t ld,
                                                      const int32_t* __restrict__ count,
                                                      const float2* __restrict__ CU,
                                                      const float2* __restrict__ V,
                                                      float2* __restrict__ G) {
  const int K = *count;
  if (K == 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * (64 * TM) + (w >> 1) * (32 * TM);
  const int n = blockIdx.x * 64 + (w & 1) * 32 + (lane & 31);
  const int h = lane >> 5;
  f32x16 X[TM], Y[TM], Z[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int r = m0 + 32 * t + 8 * (e >> 2) + 4 * h + (e & 3);
      const float2 gv = r < M ? G[(int64_t)r * ld + n] : make_float2(0.f, 0.f);
      X[t][e] = gv.x;
      if (THREE_MULT) {
        Y[t][e] = 0.f;
        Z[t][e] = gv.x + gv.y;
      } else {
        Y[t][e] = gv.y;
      }
    }
  }
#pragma unroll 2
  for (int k0 = 0; k0 < K; k0 += 2) {
    const int kk = k0 + h;
    float2 a[TM], b = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < TM; ++t) a[t] = make_float2(0.f, 0.f);
    if (kk < K) {
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const int am = m0 + 32 * t + (lane & 31);
        if (am < M) a[t] = CU[(int64_t)kk * R + am];
      }
      b = V[(int64_t)kk * ld + n];
    }
    if (THREE_MULT) {
      const float bs = b.x + b.y;
#pragma unroll
      for (int t = 0; t < TM; ++t) X[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t].x, b.x, X[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < TM; ++t) Y[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t].y, b.y, Y[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < TM; ++t)
        Z[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t].x + a[t].y, bs, Z[t], 0, 0, 0);
    } else {
#pragma unroll
      for (int t = 0; t < TM; ++t) X[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t].x, b.x, X[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < TM; ++t) Y[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t].x, b.y, Y[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < TM; ++t) X[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[t].y, b.y, X[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < TM; ++t) Y[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t].y, b.x, Y[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < TM; ++t) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int r = m0 + 32 * t + 8 * (e >> 2) + 4 * h + (e & 3);
      if (r >= M) continue;
      const float2 out = THREE_MULT ? make_float2(X[t][e] - Y[t][e], Z[t][e] - X[t][e] - Y[t][e])
                                    : make_float2(X[t][e], Y[t][e]);
      G[(int64_t)r * ld + n] = out;
    }
  }
}

// Prefetching variant, 32 x 32 per wave and 64 x 64 per workgroup: every CU and
// V operand of the wave (all GFO_MAX_DELAY slots, 32 instruction steps; slots
// past the pending count contribute zero) is loaded into registers first, then
// the wave's G tile is requested, and the products accumulate from zero while
// the G loads are in flight; G is added in the epilogue.  Vector loads complete
// in issue order, so the operands are ready without waiting for G.  A partial
// flush costs as much as a full one.  Byte offsets are 32-bit: the launcher uses
// this form only when GFO_MAX_DELAY * max(R, ld) * 8 < 2^31.  THREE_MULT as in
// k_flush_c64_tm.
template <bool THREE_MULT>
__global__ __launch_bounds__(256) void k_flush_c64_pf(int M, int R, int64_t ld,
                                                      const int32_t* __restrict__ count,
                                                      const float2* __restrict__ CU,
                                                      const float2* __restrict__ V,
                                                      float2* __restrict__ G) {
  const int K = *count;
  if (K == 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int n = blockIdx.x * 64 + (w & 1) * 32 + (lane & 31);
  const int h = lane >> 5;
  const int am = m0 + (lane & 31);
  constexpr int P = GFO_MAX_DELAY / 2;           // instruction steps (two terms each)
  // Operands come through buffer loads whose range ends at the pending count, so
  // the slots past it (and rows past the end, given an offset beyond the range)
  // read as zero without a branch or a select: the first product then waits only
  // for the operand loads, not for the G loads issued after them.
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc((void*)CU, (short)0, K * R * 8, kBufferDword3);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc((void*)V, (short)0, (int)(K * ld * 8), kBufferDword3);
  const unsigned a_off = am < M ? (unsigned)(h * R + am) * 8u : 0xFFFFFFF0u;
  const unsigned b_off = (unsigned)(h * ld + n) * 8u;
  float2 a[P], b[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const unsigned da = am < M ? (unsigned)(2 * i) * (unsigned)R * 8u : 0u;
    const auto va = __builtin_amdgcn_raw_buffer_load_b64(ra, a_off + da, 0, 0);
    const auto vb = __builtin_amdgcn_raw_buffer_load_b64(rb, b_off + (unsigned)(2 * i * ld) * 8u, 0, 0);
    const f32x2 fa = __builtin_bit_cast(f32x2, va), fb = __builtin_bit_cast(f32x2, vb);
    a[i] = make_float2(fa[0], fa[1]);
    b[i] = make_float2(fb[0], fb[1]);
  }
  // keep the issue order (operands, then G, then products): the scheduler would
  // otherwise sink the loads next to their first use
  __builtin_amdgcn_sched_barrier(0);
  float2 gv[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int r = m0 + 8 * (e >> 2) + 4 * h + (e & 3);
    gv[e] = G[(int64_t)(r < M ? r : M - 1) * ld + n];
  }
  __builtin_amdgcn_sched_barrier(0);
  f32x16 X, Y, Z;
#pragma unroll
  for (int e = 0; e < 16; ++e) X[e] = Y[e] = Z[e] = 0.f;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    if (THREE_MULT) {
      X = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[i].x, X, 0, 0, 0);
      Y = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[i].y, Y, 0, 0, 0);
      Z = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x + a[i].y, b[i].x + b[i].y, Z, 0, 0, 0);
    } else {
      X = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[i].x, X, 0, 0, 0);
      Y = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].x, b[i].y, Y, 0, 0, 0);
      X = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[i].y, b[i].y, X, 0, 0, 0);
      Y = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i].y, b[i].x, Y, 0, 0, 0);
    }
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int r = m0 + 8 * (e >> 2) + 4 * h + (e & 3);
    if (r >= M) continue;
    const float2 out = THREE_MULT ? make_float2(gv[e].x + (X[e] - Y[e]), gv[e].y + (Z[e] - X[e] - Y[e]))
                                  : make_float2(gv[e].x + X[e], gv[e].y + Y[e]);
    G[(int64_t)r * ld + n] = out;
  }
}

// Software-pipelined form of k_flush_c64_pf: registers hold the operands of 16
// instruction steps (half the slots); the G tile is requested after the first
// 16, and each register is reloaded with the operands 16 steps ahead as soon as
// its step is consumed.  Same ranged buffer loads (empty slots read as zero), and
// the same 32-bit offset limit.
template <bool THREE_MULT>
__global__ __launch_bounds__(256) void k_flush_c64_pipe(int M, int R, int64_t ld,
                                                        const int32_t* __restrict__ count,
                                                        const float2* __restrict__ CU,
                                                        const float2* __restrict__ V,
                                                        float2* __restrict__ G) {
  const int K = *count;
  if (K == 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int n = blockIdx.x * 64 + (w & 1) * 32 + (lane & 31);
  const int h = lane >> 5;
  const int am = m0 + (lane & 31);
  constexpr int P = GFO_MAX_DELAY / 2, H = P / 2;
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc((void*)CU, (short)0, K * R * 8, kBufferDword3);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc((void*)V, (short)0, (int)(K * ld * 8), kBufferDword3);
  const unsigned a_off = am < M ? (unsigned)(h * R + am) * 8u : 0xFFFFFFF0u;
  const unsigned a_step = am < M ? 2u * (unsigned)R * 8u : 0u;
  const unsigned b_off = (unsigned)(h * ld + n) * 8u, b_step = 2u * (unsigned)ld * 8u;
  f32x2 a[H], b[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    a[i] = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(ra, a_off + i * a_step, 0, 0));
    b[i] = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rb, b_off + i * b_step, 0, 0));
  }
  __builtin_amdgcn_sched_barrier(0);
  float2 gv[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int r = m0 + 8 * (e >> 2) + 4 * h + (e & 3);
    gv[e] = G[(int64_t)(r < M ? r : M - 1) * ld + n];
  }
  __builtin_amdgcn_sched_barrier(0);
  f32x16 X, Y, Z;
#pragma unroll
  for (int e = 0; e < 16; ++e) X[e] = Y[e] = Z[e] = 0.f;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const f32x2 ai = a[i % H], bi = b[i % H];
    if (i < H) {
      a[i] = __builtin_bit_cast(f32x2,
                                __builtin_amdgcn_raw_buffer_load_b64(ra, a_off + (i + H) * a_step, 0, 0));
      b[i] = __builtin_bit_cast(f32x2,
                                __builtin_amdgcn_raw_buffer_load_b64(rb, b_off + (i + H) * b_step, 0, 0));
    }
    if (THREE_MULT) {
      X = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[0], bi[0], X, 0, 0, 0);
      Y = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[1], bi[1], Y, 0, 0, 0);
      Z = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[0] + ai[1], bi[0] + bi[1], Z, 0, 0, 0);
    } else {
      X = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[0], bi[0], X, 0, 0, 0);
      Y = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[0], bi[1], Y, 0, 0, 0);
      X = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai[1], bi[1], X, 0, 0, 0);
      Y = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[1], bi[0], Y, 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int r = m0 + 8 * (e >> 2) + 4 * h + (e & 3);
    if (r >= M) continue;
    const float2 out = THREE_MULT ? make_float2(gv[e].x + (X[e] - Y[e]), gv[e].y + (Z[e] - X[e] - Y[e]))
                                  : make_float2(gv[e].x + X[e], gv[e].y + Y[e]);
    G[(int64_t)r * ld + n] = out;
  }
}

// flush variants for complex64 storage (selected by the autotuner)
static std::atomic<int> g_flush_sel{0};
static const char* const kFlushNames[] = {"w32", "w64_xcd", "w32x2", "w32_3m", "w32x2_3m", "w32_pf", "w32_pf_3m", "w32_pipe", "w32_pipe_3m"};
constexpr int kFlushCount = (int)(sizeof(kFlushNames) / sizeof(kFlushNames[0]));
int flush_variant_count() { return kFlushCount; }
const char* flush_variant_name(int i) { return i >= 0 && i < kFlushCount ? kFlushNames[i] : nullptr; }
int flush_set_variant(int i) {
  if (i < 0 || i >= kFlushCount) return GFO_EINVAL;
  g_flush_sel.store(i);
  return GFO_OK;
}
int flush_get_variant() { return g_flush_sel.load(); }

__global__ void k_dl_reset(int32_t* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count = 0;
}

hipError_t launch_dl_reset(const Geo&, gfo_state* st, const Layout& L, hipStream_t s) {
  hipLaunchKernelGGL(k_dl_reset, dim3(1), dim3(64), 0, s, (int32_t*)((char*)st->work + L.dl_hdr));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_deferred(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                                 hipStream_t s) {
  char* w = (char*)st->work;
  Snap* snap = (Snap*)(w + L.snap);
  int32_t* count = (int32_t*)(w + L.dl_hdr);
  T* cu = (T*)(w + L.cu);
  T* v = (T*)(w + L.v);
  const int64_t n = (int64_t)g.R + g.ld;
  hipLaunchKernelGGL(k_gather_dl<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, pick,
                     (const T*)st->G, (const T*)st->E, (const double2*)st->diag64,
                     (const uint8_t*)st->eps_idx, (const int32_t*)count, snap, (T*)(w + L.dl_CU),
                     (T*)(w + L.dl_V), (T*)(w + L.dl_CUs), (T*)(w + L.dl_Vs), cu, v);
  const int64_t nx = g.R > g.ld ? (int64_t)g.R : g.ld;
  dim3 gm((unsigned)((nx + 255) / 256), (unsigned)(g.nmon < 65535 ? g.nmon : 65535));
  hipLaunchKernelGGL(k_mon_dl<T>, gm, dim3(256), 0, s, g, (const Snap*)snap, (const T*)cu,
                     (const T*)v, (T*)st->G, (T*)st->E, (double2*)st->diag64, st->eps_idx, st->flips,
                     st->flip_cap, st->n_flips, st->status, count);
  return hipGetLastError();
}
template hipError_t launch_apply_deferred<float2>(const Geo&, gfo_state*, const Layout&,
                                                  const gfo_pick*, hipStream_t);
template hipError_t launch_apply_deferred<double2>(const Geo&, gfo_state*, const Layout&,
                                                   const gfo_pick*, hipStream_t);

hipError_t launch_flush(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s) {
  char* w = (char*)st->work;
  const int32_t* count = (const int32_t*)(w + L.dl_hdr);
  hipEvent_t before, after;
  k1_take_timing(&before, &after);
  hipError_t e;
  if (g.dtype == GFO_C64) {
    if (before && hipEventRecord(before, s) != hipSuccess) return hipErrorUnknown;
    const int fv = flush_get_variant();
    const float2* cu = (const float2*)(w + L.dl_CUs);
    const float2* vv = (const float2*)(w + L.dl_Vs);
    const dim3 g1((unsigned)(g.ld / 64), (unsigned)((g.N + 63) / 64));
    const dim3 g2((unsigned)(g.ld / 64), (unsigned)((g.N + 127) / 128));
    if (fv == 2) {
      hipLaunchKernelGGL((k_flush_c64_tm<2, false>), g2, dim3(256), 0, s, g.N, g.R, g.ld, count, cu, vv,
                         (float2*)st->G);
    } else if (fv == 3) {
      hipLaunchKernelGGL((k_flush_c64_tm<1, true>), g1, dim3(256), 0, s, g.N, g.R, g.ld, count, cu, vv,
                         (float2*)st->G);
    } else if (fv == 4) {
      hipLaunchKernelGGL((k_flush_c64_tm<2, true>), g2, dim3(256), 0, s, g.N, g.R, g.ld, count, cu, vv,
                         (float2*)st->G);
    } else if (fv >= 5 && fv <= 8 &&
               (int64_t)GFO_MAX_DELAY * (g.ld > g.R ? g.ld : g.R) * 8 >= ((int64_t)1 << 31)) {
      return hipErrorInvalidValue;
    } else if (fv == 5) {
      hipLaunchKernelGGL((k_flush_c64_pf<false>), g1, dim3(256), 0, s, g.N, g.R, g.ld, count, cu, vv,
                         (float2*)st->G);
    } else if (fv == 6) {
      hipLaunchKernelGGL((k_flush_c64_pf<true>), g1, dim3(256), 0, s, g.N, g.R, g.ld, count, cu, vv,
                         (float2*)st->G);
    } else if (fv == 7) {
      hipLaunchKernelGGL((k_flush_c64_pipe<false>), g1, dim3(256), 0, s, g.N, g.R, g.ld, count, cu, vv,
                         (float2*)st->G);
    } else if (fv == 8) {
      hipLaunchKernelGGL((k_flush_c64_pipe<true>), g1, dim3(256), 0, s, g.N, g.R, g.ld, count, cu, vv,
                         (float2*)st->G);
    } else if (fv == 0) {
      hipLaunchKernelGGL(k_flush_c64, dim3((unsigned)(g.ld / 64), (unsigned)((g.N + 63) / 64)),
                         dim3(256), 0, s, g.N, g.R, g.ld, count, (const float2*)(w + L.dl_CUs),
                         (const float2*)(w + L.dl_Vs), (float2*)st->G);
    } else {
      const int nbx = (int)((g.ld + 127) / 128), nby = (g.N + 127) / 128;
      const int per = (nbx * nby + 7) / 8;
      hipLaunchKernelGGL(k_flush_c64_w64, dim3((unsigned)(per * 8)), dim3(256), 0, s, g.N, g.R, g.ld,
                         nbx, nby, count, (const float2*)(w + L.dl_CUs), (const float2*)(w + L.dl_Vs),
                         (float2*)st->G);
    }
    e = hipGetLastError();
  } else {
    if (before && hipEventRecord(before, s) != hipSuccess) return hipErrorUnknown;
    e = launch_zgemm_update_f64(g, count, (const double2*)(w + L.dl_CUs),
                                (const double2*)(w + L.dl_Vs), (double2*)st->G, s);
  }
  if (e != hipSuccess) return e;
  if (after && hipEventRecord(after, s) != hipSuccess) return hipErrorUnknown;
  hipLaunchKernelGGL(k_dl_reset, dim3(1), dim3(64), 0, s, (int32_t*)(w + L.dl_hdr));
  return hipGetLastError();
}

}  // namespace gfo
