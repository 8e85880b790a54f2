// The flush of the deferred rank-1 terms: G[m, n] += sum_{s < count} CU[s][m] V[s][n]
// (eq. form10, grouped) on the matrix cores, for the design block and the
// monitor rows other than the FOM monitor's, and the copy of the design block's
// upper triangle into its lower one.  Complex64 variants are selected by the
// autotuner; complex128 storage uses the FP64 GEMM.
#include "gfo_internal.hpp"

#include <atomic>
#include <type_traits>

namespace gfo {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Fourth word of a raw buffer resource on gfx9-family chips (32-bit data format;
// reads past the range return zero).
constexpr int kBufferDword3 = 0x00020000;

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
                                                      float2* __restrict__ G, int row0) {
  const int K = *count;
  if (K == 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = row0 + blockIdx.y * (64 * TM) + (w >> 1) * (32 * TM);
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

// Tile t (row-major) of the triangle of nb x nb tiles on and above the
// diagonal: row r starts at tile r nb - r (r - 1) / 2.
__device__ __forceinline__ void tri_tile(int t, int nb, int& r, int& c) {
  auto start = [nb](int i) { return i * nb - i * (i - 1) / 2; };
  const double b2 = 2.0 * nb + 1.0;
  int i = (int)((b2 - sqrt(b2 * b2 - 8.0 * t)) * 0.5);
  i = i < 0 ? 0 : (i > nb - 1 ? nb - 1 : i);
  while (i > 0 && start(i) > t) --i;
  while (i < nb - 1 && start(i + 1) <= t) ++i;
  r = i;
  c = i + (t - start(i));
}

// Pair-interleaved copy of the pending terms (complex64): slots 2p and 2p + 1 of
// index i side by side, CU2[p R + i] = (CU_2p[i], CU_2p+1[i]) and likewise V2
// with ld, zero past the count, so that one 16-byte load brings a lane the
// operands of two matrix steps.  Grid: x over max(R, ld) / 256, y over the pairs.
__global__ __launch_bounds__(256) void k_flush_pack(int R, int64_t ld,
                                                    const int32_t* __restrict__ count,
                                                    const float2* __restrict__ CU,
                                                    const float2* __restrict__ V,
                                                    f32x4* __restrict__ CU2, f32x4* __restrict__ V2) {
  const int K = *count;
  const int p = (int)blockIdx.y;
  if (2 * p >= K) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool second = 2 * p + 1 < K;
  if (i < R) {
    const float2 a = CU[(int64_t)(2 * p) * R + i];
    const float2 b = second ? CU[(int64_t)(2 * p + 1) * R + i] : make_float2(0.f, 0.f);
    CU2[(int64_t)p * R + i] = f32x4{a.x, a.y, b.x, b.y};
  }
  if (i < ld) {
    const float2 a = V[(int64_t)(2 * p) * ld + i];
    const float2 b = second ? V[(int64_t)(2 * p + 1) * ld + i] : make_float2(0.f, 0.f);
    V2[(int64_t)p * ld + i] = f32x4{a.x, a.y, b.x, b.y};
  }
}

// Base offset and row stride of the 64-row tile at rows [rbase, rbase + 64),
// columns [64 bx, 64 bx + 64): a design tile (rbase < M, rbase a multiple of
// 64) in dense or band-packed storage (g_off), or a monitor tile (rows from
// M on, ld apart after mon_base).
struct TileAt {
  int64_t base, stride;
};
__device__ __forceinline__ TileAt tile_at(int packed, int M, int64_t ld, int64_t mon_base, int rbase,
                                          int bx) {
  if (rbase >= M) return TileAt{mon_base + (int64_t)(rbase - M) * ld + 64 * (int64_t)bx, ld};
  const int64_t b = rbase >> 6;
  return TileAt{g_band_start(packed, ld, b) + 64 * (bx - (packed ? b : 0)), g_band_stride(packed, ld, b)};
}

// Upper-triangle flush of the design block, three real products per complex
// one (as in k_flush_c64_tm), 32 x 32 outputs per wave, 64 x 64 per workgroup.
//
// Symmetry: the design block is symmetric (reciprocity: G_D = G_D^T, and each
// pending term restricted to it, c_s v_s v_s^T, is symmetric too), so only the
// tiles on and above the diagonal are computed: a one-dimensional grid, tile t
// in row-major order over that triangle (nby = design blocks).  The upper
// triangle alone is brought up to date; the lower tiles are left as they are
// (the caller records that the lower triangle is out of date, and readers take
// design entries from the upper one).  Diagonal tiles are computed whole,
// their lower halves from the old values.
//
// Operands: pair-interleaved terms (k_flush_pack).  In pair step m, lane (row
// or column, h) loads pair 2m + h, i.e. slots 4m + 2h and 4m + 2h + 1, and
// feeds them to two matrix steps (the instruction sums its two k lanes, here
// slots 4m + 2h' for h' = 0, 1 in the first step and 4m + 2h' + 1 in the
// second).  The operands come through buffer loads whose range ends at the
// pending count, so slots past it (and rows past the end, given an offset
// beyond the range) read as zero without a branch or a select.  HP pair steps
// of operands in registers (a ring, each entry reloaded HP steps ahead); PP
// pair steps per launch, the fewest of 4, 8, 16 and 32 (16 to 128 terms) that
// cover the caller's bound on the count.  Byte offsets are 32-bit: the
// launcher uses this form only when GFO_MAX_DELAY * max(R, ld) * 8 < 2^31.
//
// G is read and written with non-temporal (streaming) loads and stores; the
// operand terms, which every workgroup re-reads, keep the normal policy.  The
// products accumulate from zero and G is added in the epilogue.  Ring depths
// of 2 and 8 pair steps measured no faster (8 drops to two waves per SIMD),
// nor did moving the G tile in 16-byte pieces (adjacent lanes exchanging
// halves).
//
// The workgroups past the nby (nby + 1) / 2 triangle tiles take the monitor
// rows [M, R) in 64 x 64 tiles over all ld columns (the FOM monitor's terms
// are zeros, and G is added in the epilogue, so its row is rewritten unchanged).
// XORD: the XCD tile order (xcd_tile): the grid is 8 x the largest per-XCD
// tile count, and workgroups without a tile return at once.
template <int HP, int PP, bool XORD = false>
__global__ __launch_bounds__(256) void k_flush_c64_pair(int M, int R, int64_t ld,
                                                        const int32_t* __restrict__ count,
                                                        const f32x4* __restrict__ CU2,
                                                        const f32x4* __restrict__ V2,
                                                        float2* __restrict__ G, int nby,
                                                        int packed, int64_t mon_base) {
  const int K = *count;
  if (K == 0) return;
  const int ntri = nby * (nby + 1) / 2;
  int by, bx, lim, rbase;
  if constexpr (XORD) {
    const int nbx = (int)(ld / 64), nmb = (R - M + 63) / 64;
    bool mon = false;
    if (!xcd_tile((int)blockIdx.x, nby, nbx, nmb, &by, &bx, &mon)) return;
    if (bx < 0 || bx >= nbx || by < 0 || by >= (mon ? nmb : nby)) return;
    lim = mon ? R : M;
    rbase = mon ? M + by * 64 : by * 64;
  } else if ((int)blockIdx.x < ntri) {
    tri_tile((int)blockIdx.x, nby, by, bx);
    lim = M;
    rbase = by * 64;
  } else {
    const int t = (int)blockIdx.x - ntri, nbx = (int)(ld / 64);
    bx = t % nbx;
    lim = R;
    rbase = M + (t / nbx) * 64;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = rbase + (w >> 1) * 32;
  const int n = bx * 64 + (w & 1) * 32 + (lane & 31);
  const int h = lane >> 5;
  const int am = m0 + (lane & 31);
  static_assert(PP % HP == 0, "ring depth divides the pair-step count");
  const int np = (K + 1) / 2;
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc((void*)CU2, (short)0, np * R * 16, kBufferDword3);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc((void*)V2, (short)0, (int)(np * ld * 16), kBufferDword3);
  const unsigned a_off = am < lim ? (unsigned)(h * R + am) * 16u : 0xFFFFFFF0u;
  const unsigned a_step = am < lim ? 2u * (unsigned)R * 16u : 0u;
  const unsigned b_off = (unsigned)(h * ld + n) * 16u, b_step = 2u * (unsigned)ld * 16u;
  f32x4 a[HP], b[HP];
#pragma unroll
  for (int i = 0; i < HP; ++i) {
    a[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, a_off + i * a_step, 0, 0));
    b[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, b_off + i * b_step, 0, 0));
  }
  __builtin_amdgcn_sched_barrier(0);
  // the tile in G (dense or band-packed design rows, monitor rows)
  const TileAt ta = tile_at(packed, M, ld, mon_base, rbase, bx);
  float2* __restrict__ Gt = G + ta.base + (n - bx * 64);
  float2 gv[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int r = m0 + 8 * (e >> 2) + 4 * h + (e & 3);
    const float2* src = Gt + (int64_t)((r < lim ? r : lim - 1) - rbase) * ta.stride;
    gv[e] = __builtin_bit_cast(float2, __builtin_nontemporal_load((const f32x2*)src));
  }
  __builtin_amdgcn_sched_barrier(0);
  f32x16 X, Y, Z;
#pragma unroll
  for (int e = 0; e < 16; ++e) X[e] = Y[e] = Z[e] = 0.f;
#pragma unroll
  for (int i = 0; i < PP; ++i) {
    const f32x4 ai = a[i % HP], bi = b[i % HP];
    if (i + HP < PP) {
      a[i % HP] = __builtin_bit_cast(
          f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, a_off + (i + HP) * a_step, 0, 0));
      b[i % HP] = __builtin_bit_cast(
          f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, b_off + (i + HP) * b_step, 0, 0));
    }
    X = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[0], bi[0], X, 0, 0, 0);
    Y = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[1], bi[1], Y, 0, 0, 0);
    Z = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[0] + ai[1], bi[0] + bi[1], Z, 0, 0, 0);
    X = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[2], bi[2], X, 0, 0, 0);
    Y = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[3], bi[3], Y, 0, 0, 0);
    Z = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[2] + ai[3], bi[2] + bi[3], Z, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int r = m0 + 8 * (e >> 2) + 4 * h + (e & 3);
    if (r < lim) {
      const float2 out = make_float2(gv[e].x + (X[e] - Y[e]), gv[e].y + (Z[e] - X[e] - Y[e]));
      __builtin_nontemporal_store(f32x2{out.x, out.y}, (f32x2*)(Gt + (int64_t)(r - rbase) * ta.stride));
    }
  }
}


typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Position of a persistent flush run in the tile list in column segments of sw
// tiles (segment j: columns [sw j, sw j + sw)); inside a segment the triangle's
// rows top to bottom, then the monitor bands, each row left to right.
struct SegTile {
  int band, bx, lim, rbase, seg;
};
struct SegWalk {
  int M, R, nby, nbx, nmb, sw;   // sw: segment width in tiles
  __device__ int seg_tri(int j) const {
    const int s0 = sw * j;
    if (s0 >= nby) return 0;
    const int wd = (s0 + sw < nby ? s0 + sw : nby) - s0;
    return s0 * wd + wd * (wd + 1) / 2;
  }
  __device__ int seg_mon(int j) const {
    const int s0 = sw * j;
    return nmb * ((s0 + sw < nbx ? s0 + sw : nbx) - s0);
  }
  __device__ SegTile at(int t) const {
    SegTile c{0, 0, M, 0, 0};
    int u = t;
    while (u >= seg_tri(c.seg) + seg_mon(c.seg)) {
      u -= seg_tri(c.seg) + seg_mon(c.seg);
      ++c.seg;
    }
    const int s0 = sw * c.seg, nt = seg_tri(c.seg);
    if (u < nt) {
      const int e = s0 + sw < nby ? s0 + sw : nby, wd = e - s0;
      if (u < s0 * wd) {
        c.band = u / wd;
        c.bx = s0 + u % wd;
      } else {
        u -= s0 * wd;
        c.band = s0;
        while (u >= e - c.band) {
          u -= e - c.band;
          ++c.band;
        }
        c.bx = c.band + u;
      }
      c.rbase = c.band * 64;
    } else {
      u -= nt;
      const int wd = (s0 + sw < nbx ? s0 + sw : nbx) - s0;
      c.band = nby + u / wd;
      c.bx = s0 + u % wd;
      c.lim = R;
      c.rbase = M + (u / wd) * 64;
    }
    return c;
  }
  // the tile after c (c itself when the list ends there)
  __device__ SegTile next(const SegTile& c) const {
    SegTile n = c;
    const int s0 = sw * c.seg;
    bool next_seg = false;
    if (c.band < nby) {
      const int e = s0 + sw < nby ? s0 + sw : nby;
      if (c.bx + 1 < e) {
        n.bx = c.bx + 1;
      } else if (c.band + 1 < e) {
        n.band = c.band + 1;
        n.bx = n.band > s0 ? n.band : s0;
        n.rbase = n.band * 64;
      } else if (nmb > 0) {
        n.band = nby;
        n.bx = s0;
        n.lim = R;
        n.rbase = M;
      } else {
        next_seg = true;
      }
    } else {
      const int f = s0 + sw < nbx ? s0 + sw : nbx;
      if (c.bx + 1 < f) {
        n.bx = c.bx + 1;
      } else if (c.band + 1 < nby + nmb) {
        n.band = c.band + 1;
        n.bx = s0;
        n.rbase = c.rbase + 64;
      } else {
        next_seg = true;
      }
    }
    if (next_seg) {
      if (s0 + sw >= nbx) return c;
      n.seg = c.seg + 1;
      n.bx = s0 + sw;
      if (n.bx < nby) {
        n.band = 0;
        n.lim = M;
        n.rbase = 0;
      } else {
        n.band = nby;
        n.lim = R;
        n.rbase = M;
      }
    }
    return n;
  }
};

// The same list in row-major order: the triangle's rows top to bottom, each
// left to right, then the monitor bands.
struct RowWalk {
  int M, R, nby, nbx, nmb;
  __device__ SegTile at(int t) const {
    SegTile c{0, 0, M, 0, 0};
    const int ntri = nby * (nby + 1) / 2;
    if (t < ntri) {
      tri_tile(t, nby, c.band, c.bx);
      c.rbase = c.band * 64;
    } else {
      const int u = t - ntri;
      c.bx = u % nbx;
      c.band = nby + u / nbx;
      c.lim = R;
      c.rbase = M + (u / nbx) * 64;
    }
    return c;
  }
  // the tile after c (the caller asks only while one follows)
  __device__ SegTile next(const SegTile& c) const {
    SegTile n = c;
    if (c.band < nby) {
      if (c.bx + 1 < nby) {
        n.bx = c.bx + 1;
      } else if (c.band + 1 < nby) {
        n.band = c.band + 1;
        n.bx = n.band;
        n.rbase = n.band * 64;
      } else {
        n.band = nby;
        n.bx = 0;
        n.lim = R;
        n.rbase = M;
      }
    } else if (c.bx + 1 < nbx) {
      n.bx = c.bx + 1;
    } else {
      n.band = c.band + 1;
      n.bx = 0;
      n.rbase = c.rbase + 64;
    }
    return n;
  }
};

// Persistent form of the pair flush (same operands, same matrix steps in the same
// order, so the same results bit for bit): workgroup b takes a contiguous run of
// the tile list (triangle tiles row by row, then the monitor rows' tiles; runs in
// XCD order, workgroup b on XCD b % 8 taking run (b % 8) P/8 + b / 8).  Per wave:
// the CU operands of its 32 rows of the current row band stay in registers
// (reloaded when the run enters a new band); the V operands of a tile go
// through LDS, one copy per workgroup; the G tile is read two tiles ahead, in
// two register sets that alternate between tiles.  Per tile the loads are
// issued in the order V(t+1), G(t+1), so the wait for V(t+1) at the end of tile
// t leaves G(t+1) in flight and the matrix loop never waits on memory.  G is
// read and written through a buffer whose range ends at the tile's last row
// (rows past the matrix read zero, their stores are dropped).  Odd runs start
// by sleeping for about half a tile, so that the two workgroups sharing a
// compute unit reach their epilogues at different times.
//
// SEGO: the tile list in column segments of 32 tiles (segment j: columns
// [32 j, 32 j + 32)), inside a segment the triangle rows top to bottom, then the
// monitor bands, each row left to right.  The runs of one XCD then share a
// segment's V operands (1 MB at 64 terms), which stay in its L2; the CU operands
// change at each row, once per at most 32 tiles.
template <int PP, bool SEGO>
__global__ __launch_bounds__(256) void k_flush_c64_band(int M, int R, int64_t ld,
                                                        const int32_t* __restrict__ count,
                                                        const f32x4* __restrict__ CU2,
                                                        const f32x4* __restrict__ V2,
                                                        float2* __restrict__ G, int nby, int chunk,
                                                        int packed, int64_t mon_base) {
  const int K = *count;
  if (K == 0) return;
  const int ntri = nby * (nby + 1) / 2;
  const int nbx = (int)(ld / 64), nmb = (R - M + 63) / 64;
  const int T = ntri + nmb * nbx;
  const int P = (int)gridDim.x, b = (int)blockIdx.x;
  const int run = (P & 7) == 0 ? (b & 7) * (P >> 3) + (b >> 3) : b;
  const int t0 = run * chunk;
  const int t1 = t0 + chunk < T ? t0 + chunk : T;
  if (t0 >= t1) return;
  __shared__ f32x4 Vsh[2 * PP][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int np = (K + 1) / 2;
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc((void*)CU2, (short)0, np * R * 16, kBufferDword3);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc((void*)V2, (short)0, (int)(np * ld * 16), kBufferDword3);
  const int q = (w >> 1) * 32 + (lane & 31);   // row of the band (CU operand)
  const int cc = (w & 1) * 32 + (lane & 31);  // column of the tile (V operand)
  const int lrow = (w >> 1) * 32 + 4 * h;     // the lane's first row within a tile
  f32x4 aR[PP];
  auto load_A = [&](int lim, int rbase) {
    const int am = rbase + q;
    const unsigned off = am < lim ? (unsigned)(h * R + am) * 16u : 0xFFFFFFF0u;
    const unsigned st = am < lim ? 2u * (unsigned)R * 16u : 0u;
#pragma unroll
    for (int i = 0; i < PP; ++i)
      aR[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, off + i * st, 0, 0));
  };
  constexpr int NB = (2 * PP * 64) / 256;
  f32x4 bs[NB];
  auto load_B = [&](int bx) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = j * 256 + (int)threadIdx.x;
      const unsigned off = (unsigned)((e >> 6) * ld + bx * 64 + (e & 63)) * 16u;
      bs[j] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, off, 0, 0));
    }
  };
  auto stage_B = [&]() {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = j * 256 + (int)threadIdx.x;
      Vsh[e >> 6][e & 63] = bs[j];
    }
  };
  // the tile's G through a buffer resource whose range ends at its last row
  // (dense or band-packed design rows: tile_at gives the row stride)
  auto g_rsrc = [&](int bx, int lim, int rbase, int64_t& stride) {
    const int rows = lim - rbase < 64 ? lim - rbase : 64;
    const TileAt ta = tile_at(packed, M, ld, mon_base, rbase, bx);
    stride = ta.stride;
    return __builtin_amdgcn_make_buffer_rsrc((void*)(G + ta.base), (short)0,
                                             (int)((int64_t)rows * ta.stride * 8), kBufferDword3);
  };
  // byte offsets: the lane's (vector) and element e's row (uniform, a scalar offset)
  auto lane_off = [&](int64_t stride) { return (unsigned)((int64_t)lrow * stride + cc) * 8u; };
  auto row_off = [&](int64_t stride, int e) { return (int)((int64_t)(8 * (e >> 2) + (e & 3)) * stride * 8); };
  auto load_G = [&](__amdgpu_buffer_rsrc_t rg, int64_t stride, float2(&gv)[16]) {
    const unsigned vo = lane_off(stride);
#pragma unroll
    for (int e = 0; e < 16; ++e)
      gv[e] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rg, vo, row_off(stride, e), 2));
  };
  // the run's tiles: column segments of 32 tiles (SEGO) or row-major order
  using Walk = typename std::conditional<SEGO, SegWalk, RowWalk>::type;
  Walk walk;
  if constexpr (SEGO) walk = SegWalk{M, R, nby, nbx, nmb, 32};
  else walk = RowWalk{M, R, nby, nbx, nmb};
  const SegTile c0 = walk.at(t0);
  int band = c0.band, bx = c0.bx, lim = c0.lim, rbase = c0.rbase, seg = c0.seg;
  float2 gA[16], gB[16];
  load_A(lim, rbase);
  load_B(bx);
  int64_t scur;
  __amdgpu_buffer_rsrc_t rcur = g_rsrc(bx, lim, rbase, scur);
  load_G(rcur, scur, gA);
  stage_B();
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the operands are in registers on every path
  __syncthreads();
  if ((run & 1) && (P & 7) == 0) __builtin_amdgcn_s_sleep(48);
  auto tile = [&](int t, float2(&gc)[16], float2(&gn)[16]) {
    // the next tile of the run (this one at the run's end)
    const SegTile nt = t + 1 < t1 ? walk.next(SegTile{band, bx, lim, rbase, seg}) : SegTile{band, bx, lim, rbase, seg};
    const int nband = nt.band, nbxx = nt.bx, nlim = nt.lim, nrbase = nt.rbase, nseg = nt.seg;
    load_B(nbxx);
    int64_t snext;
    const __amdgpu_buffer_rsrc_t rnext = g_rsrc(nbxx, nlim, nrbase, snext);
    load_G(rnext, snext, gn);
    __builtin_amdgcn_sched_barrier(0);
    f32x16 X, Y, Z;
#pragma unroll
    for (int e = 0; e < 16; ++e) X[e] = Y[e] = Z[e] = 0.f;
    f32x4 br[2];
    br[0] = Vsh[h][cc];
    br[1] = Vsh[2 + h][cc];
#pragma unroll
    for (int i = 0; i < PP; ++i) {
      const f32x4 ai = aR[i], bi = br[i & 1];
      if (i + 2 < PP) br[i & 1] = Vsh[2 * (i + 2) + h][cc];
      X = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[0], bi[0], X, 0, 0, 0);
      Y = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[1], bi[1], Y, 0, 0, 0);
      Z = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[0] + ai[1], bi[0] + bi[1], Z, 0, 0, 0);
      X = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[2], bi[2], X, 0, 0, 0);
      Y = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[3], bi[3], Y, 0, 0, 0);
      Z = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[2] + ai[3], bi[2] + bi[3], Z, 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    const unsigned vo = lane_off(scur);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const f32x2 o = {gc[e].x + (X[e] - Y[e]), gc[e].y + (Z[e] - X[e] - Y[e])};
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, o), rcur, vo, row_off(scur, e), 2);
    }
    __syncthreads();  // every wave is done with this tile's V operands
    stage_B();
    __syncthreads();
    if (nband != band) {
      load_A(nlim, nrbase);
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    band = nband;
    bx = nbxx;
    lim = nlim;
    rbase = nrbase;
    seg = nseg;
    rcur = rnext;
    scur = snext;
  };
  for (int t = t0; t < t1; t += 2) {
    tile(t, gA, gB);
    if (t + 1 >= t1) break;
    tile(t + 1, gB, gA);
  }
}


// ---------------------------------------------------------------------------
// Split-product flush: the FP32 products on the BF16 matrix cores.  Each FP32
// operand x is split into three BF16 parts, x = x0 + x1 + x2 + r (x0 the
// nearest BF16 to x, x1 to x - x0, x2 to x - x0 - x1; every difference is exact
// in FP32; with u = 2^-8 the unit roundoff of BF16, |x1| <= u |x|, |x2| <= u^2 |x|
// and |r| <= u^3 |x| = 2^-24 |x|), and a product a b is summed from the six part
// products a_i b_j with i + j <= 2.  Each part product is exact in FP32 and the
// matrix core accumulates in FP32; the dropped part products and the residuals
// come to about 4 u^3 |a||b|, a few units of FP32 rounding, so the sum has FP32
// accuracy.  v_mfma_f32_32x32x16_bf16 takes 16 terms in 32 cycles
// where v_mfma_f32_32x32x2f32 takes 2 in 64: with six part products and four
// real products per complex one, a term costs half the matrix-core cycles of
// the three-product FP32 form.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split3(float x, __bf16& x0, __bf16& x1, __bf16& x2) {
  x0 = (__bf16)x;
  const float r1 = x - (float)x0;
  x1 = (__bf16)r1;
  x2 = (__bf16)(r1 - (float)x1);
}

// Split planes of the pending terms.  Unit u = 6 (2 c + h) + p holds, for each
// index i, slots 16 c + 8 h + j (j < 8) of plane p: 0-2 the parts of the real
// part, 3-5 those of the imaginary part; 16 bytes, zero past the count.
// A3[u R + i] from CU (i < R), V3[u ld + i] from V (i < ld).  Grid: x over
// max(R, ld) / 256, y over the 2 KC (c, h) groups.
template <int KC>
__global__ __launch_bounds__(256) void k_flush_pack_s3(int R, int64_t ld,
                                                       const int32_t* __restrict__ count,
                                                       const float2* __restrict__ CU,
                                                       const float2* __restrict__ V,
                                                       bf16x8* __restrict__ A3, bf16x8* __restrict__ V3) {
  const int K = *count;
  const int ch = (int)blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  auto emit = [&](const float2* src, int64_t n, bf16x8* dst) {
    if (i >= n) return;
    bf16x8 pl[6];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int s = 8 * ch + j;
      const float2 z = s < K ? src[(int64_t)s * n + i] : make_float2(0.f, 0.f);
      __bf16 a, b, c;
      split3(z.x, a, b, c);
      pl[0][j] = a;
      pl[1][j] = b;
      pl[2][j] = c;
      split3(z.y, a, b, c);
      pl[3][j] = a;
      pl[4][j] = b;
      pl[5][j] = c;
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) dst[(int64_t)(6 * ch + p) * n + i] = pl[p];
  };
  emit(CU, R, A3);
  emit(V, ld, V3);
}

// Persistent band flush with split products (KC chunks of 16 terms: 2 for up to
// 32 terms, 4 for up to 64 at two workgroups per compute unit; 8 for up to 128
// at one, its A parts taking 192 registers of a wave, its B halves 96 KB of
// LDS).  Same tile list, run assignment, G buffers and
// epilogue layout as k_flush_c64_band in column-segment order; per wave the
// output is the 32 x 32 block (rows 32 (w >> 1), columns 32 (w & 1)) of the
// tile, accumulated as XR = sum Ar Br, XI = sum Ai Bi, Z = sum (Ar Bi + Ai Br).
// Operands:
//   - A (the row band's split CU planes, 6 KC x 16 bytes per lane) stays in
//     registers while the run stays in the band;
//   - B (the tile's split V planes, 12 KC units x 64 columns) sits in LDS in two
//     halves, chunks [0, KC/2) and [KC/2, KC); each half of the next tile is
//     read into registers while the current tile's matrix steps run on the
//     other half, and written into its half after a barrier;
//   - G(t+1) is read into registers after tile t's epilogue, in flight during
//     tile t+1's matrix steps (at one workgroup per compute unit a second G
//     register set, G(t+2) in flight, measured slower: 903 against 854 us at
//     128 terms on the 128 x 128 grid).
// Global loads of one wave retire in order; the order per tile, B(t+2) first
// half, then G(t+1), lets the first-half write of the next tile wait for its
// B loads while G(t+1) is still in flight.  Rows past the matrix read zero and
// their stores are dropped (buffer ranges), so every load and store is
// unconditional.
template <int KC>
__global__ __launch_bounds__(256, KC == 8 ? 1 : 2) void k_flush_c64_s3(int M, int R, int64_t ld,
                                                      const int32_t* __restrict__ count,
                                                      const bf16x8* __restrict__ A3,
                                                      const bf16x8* __restrict__ V3,
                                                      float2* __restrict__ G, int nby, int chunk,
                                                      int packed, int64_t mon_base, int sw) {
  constexpr int NU = 12 * KC;         // split units per index
  constexpr int HU = NU / 2;          // units per LDS half
  constexpr int NS = HU * 64 / 256;   // 16-byte staging loads per thread per half
  const int K = *count;
  if (K == 0) return;
  const SegWalk walk{M, R, nby, (int)(ld / 64), (R - M + 63) / 64, sw};
  const int T = nby * (nby + 1) / 2 + walk.nmb * walk.nbx;
  const int P = (int)gridDim.x, b = (int)blockIdx.x;
  const int run = (P & 7) == 0 ? (b & 7) * (P >> 3) + (b >> 3) : b;
  const int t0 = run * chunk;
  const int t1 = t0 + chunk < T ? t0 + chunk : T;
  if (t0 >= t1) return;
  __shared__ bf16x8 Bsh[NU][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int h = lane >> 5;
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc((void*)A3, (short)0, NU * R * 16, kBufferDword3);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc((void*)V3, (short)0, (int)(NU * ld * 16), kBufferDword3);
  const int q = (w >> 1) * 32 + (lane & 31);   // row of the band (A operand)
  const int cc = (w & 1) * 32 + (lane & 31);  // column of the tile (B operand)
  const int lrow = (w >> 1) * 32 + 4 * h;     // the lane's first output row within a tile
  bf16x8 aR[6 * KC];
  auto load_A = [&](const SegTile& c) __attribute__((always_inline)) {
    const int am = c.rbase + q;
    const unsigned off = am < c.lim ? (unsigned)am * 16u : 0xFFFFFFF0u;
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const unsigned u = (unsigned)(6 * (2 * k + h) + p);
        aR[6 * k + p] = __builtin_bit_cast(
            bf16x8, __builtin_amdgcn_raw_buffer_load_b128(ra, am < c.lim ? off + u * (unsigned)R * 16u : off, 0, 0));
      }
  };
  bf16x8 S[NS];
  auto load_S = [&](int bx, int half) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int e = j * 256 + (int)threadIdx.x;
      const unsigned off = (unsigned)((int64_t)(half * HU + (e >> 6)) * ld + bx * 64 + (e & 63)) * 16u;
      S[j] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rb, off, 0, 0));
    }
  };
  auto write_S = [&](int half) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int e = j * 256 + (int)threadIdx.x;
      Bsh[half * HU + (e >> 6)][e & 63] = S[j];
    }
  };
  auto g_rsrc = [&](const SegTile& c, int64_t& stride) __attribute__((always_inline)) {
    const int rows = c.lim - c.rbase < 64 ? c.lim - c.rbase : 64;
    const TileAt ta = tile_at(packed, M, ld, mon_base, c.rbase, c.bx);
    stride = ta.stride;
    return __builtin_amdgcn_make_buffer_rsrc((void*)(G + ta.base), (short)0,
                                             (int)((int64_t)rows * ta.stride * 8), kBufferDword3);
  };
  auto lane_off = [&](int64_t stride) { return (unsigned)((int64_t)lrow * stride + cc) * 8u; };
  auto row_off = [&](int64_t stride, int e) { return (int)((int64_t)(8 * (e >> 2) + (e & 3)) * stride * 8); };
  float2 gG[16];
  auto load_G = [&](const SegTile& c, float2(&gv)[16]) __attribute__((always_inline)) {
    int64_t stride;
    const __amdgpu_buffer_rsrc_t rg = g_rsrc(c, stride);
    const unsigned vo = lane_off(stride);
#pragma unroll
    for (int e = 0; e < 16; ++e)
      gv[e] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rg, vo, row_off(stride, e), 2));
  };
  f32x16 XR, XI, Z;
  // the matrix steps of chunks [k0, k1) against the B units in LDS
  auto steps = [&](int k0, int k1) __attribute__((always_inline)) {
#pragma unroll
    for (int k = k0; k < k1; ++k) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const bf16x8 br = Bsh[6 * (2 * k + h) + j][cc];
        const bf16x8 bi = Bsh[6 * (2 * k + h) + 3 + j][cc];
#pragma unroll
        for (int i = 0; i + j < 3; ++i) {
          const bf16x8 ar = aR[6 * k + i], ai = aR[6 * k + 3 + i];
          XR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, br, XR, 0, 0, 0);
          Z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, bi, Z, 0, 0, 0);
          XI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai, bi, XI, 0, 0, 0);
          Z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ai, br, Z, 0, 0, 0);
        }
      }
    }
  };
  // prologue: tile t0's operands and B, then the next tile's first half and G(t0)
  SegTile cur = walk.at(t0);
  SegTile nxt = t0 + 1 < t1 ? walk.next(cur) : cur;
  load_A(cur);
  load_S(cur.bx, 0);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  write_S(0);
  load_S(cur.bx, 1);
  __builtin_amdgcn_s_waitcnt(0x0F70);
  write_S(1);
  load_S(nxt.bx, 0);
  load_G(cur, gG);
  __syncthreads();
  if (KC < 8 && (run & 1) && (P & 7) == 0) __builtin_amdgcn_s_sleep(48);
  for (int t = t0; t < t1; ++t) {
#pragma unroll
    for (int e = 0; e < 16; ++e) XR[e] = XI[e] = Z[e] = 0.f;
    steps(0, KC / 2);
    __syncthreads();  // every wave is done with the first half
    write_S(0);       // the next tile's first half (waits for its loads, not for G)
    load_S(nxt.bx, 1);
    steps(KC / 2, KC);
    if (nxt.band != cur.band) {
      load_A(nxt);
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    __syncthreads();  // every wave is done with the second half
    write_S(1);
    __builtin_amdgcn_sched_barrier(0);
    int64_t scur;
    const __amdgpu_buffer_rsrc_t rcur = g_rsrc(cur, scur);
    const unsigned vo = lane_off(scur);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const f32x2 o = {gG[e].x + (XR[e] - XI[e]), gG[e].y + Z[e]};
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, o), rcur, vo, row_off(scur, e), 2);
    }
    __builtin_amdgcn_sched_barrier(0);
    // B(t+2) first half, then G(t+1)
    const SegTile nn = t + 2 < t1 ? walk.next(nxt) : nxt;
    load_S(nn.bx, 0);
    load_G(nxt, gG);
    cur = nxt;
    nxt = nn;
  }
}

// flush variants for complex64 storage (selected by the autotuner; all give the
// eager results to FP32 rounding, tests/test_gpu_deferred.py).  The default,
// up_bandseg_s3: the split-product band flush for 17 to 64 terms, the pair
// flush in XCD tile order otherwise.
static const char* const kFlushNames[] = {"w32_3m", "up_pair4_3m_nt", "up_pair4_3m_nt_x8", "up_band4_3m_nt",
                                          "up_bandseg4_3m_nt", "up_bandseg_s3"};
constexpr int kFlushCount = (int)(sizeof(kFlushNames) / sizeof(kFlushNames[0]));
constexpr int kFlushDefault = 5;
static std::atomic<int> g_flush_sel{kFlushDefault};
int flush_variant_count() { return kFlushCount; }
const char* flush_variant_name(int i) { return i >= 0 && i < kFlushCount ? kFlushNames[i] : nullptr; }
int flush_set_variant(int i) {
  if (i < 0 || i >= kFlushCount) return GFO_EINVAL;
  g_flush_sel.store(i);
  return GFO_OK;
}
int flush_get_variant() { return g_flush_sel.load(); }

// Workgroups of the persistent band flush: two per compute unit (its occupancy),
// a multiple of 8 so that every XCD gets the same number of runs.
static int band_workgroups(int per_cu = 2) {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int cus = cache[dev].load();
  if (cus == 0) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    cache[dev].store(cus);
  }
  const int n = (per_cu * cus) / 8 * 8;
  return n < 8 ? 8 : n;
}

hipError_t launch_flush(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s) {
  char* w = (char*)st->work;
  const int32_t* count = (const int32_t*)(w + L.dl_hdr);
  hipEvent_t before, after;
  k1_take_timing(&before, &after);
  hipError_t e;
  if (g.dtype == GFO_C64) {
    if (hipError_t er = record_event(before, s)) return note_hip(er);
    int fv = flush_get_variant();
    bool monitors_done = false;
    // the pair and band forms address the term buffers with 32-bit byte offsets
    const bool off32 = (int64_t)GFO_MAX_DELAY * (g.ld > g.R ? g.ld : g.R) * 8 < ((int64_t)1 << 31);
    if (fv >= 1 && !off32) fv = 0;
    // band-packed storage: the pair and band forms only (they address tiles
    // through tile_at); sizes beyond their 32-bit offsets are refused
    if (g.packed) {
      if (!off32) return note_hip(hipErrorInvalidValue);
      if (fv == 0) fv = 1;
    }
    const float2* cu = (const float2*)(w + L.dl_CUs);
    const float2* vv = (const float2*)(w + L.dl_Vs);
    float2* G = (float2*)st->G;
    const dim3 grid((unsigned)(g.ld / 64), (unsigned)((g.N + 63) / 64)), blk(256);
    switch (fv) {
      case 0:
        hipLaunchKernelGGL((k_flush_c64_tm<1, true>), grid, blk, 0, s, g.N, g.R, g.ld, count, cu, vv, G,
                           0);
        break;
      default: {
        const int bound = st->pending_calls;
        // split products: 17 to 64 terms (the matrix work of up to 16 terms hides
        // behind the G stream in the pair form); 32-bit offsets into G tiles
        // split products: 17 to 128 terms (the matrix work of up to 16 terms hides
        // behind the G stream in the pair form); 32-bit offsets into G tiles and
        // into the part planes
        const int64_t nx = g.R > g.ld ? (int64_t)g.R : g.ld;
        if (fv == 5 && bound > 16 && g.ld * 64 * 8 < ((int64_t)1 << 31) &&
            (int64_t)kSplitUnits * 16 * nx < ((int64_t)1 << 31)) {
          // segments of 32 tiles up to 64 terms (16: 0.4 % less traffic, 1 % slower;
          // 64: 3.5 % more traffic), of 16 beyond (twice the V parts per column)
          const int sw = bound <= 64 ? 32 : 16;
          const int nb = (g.N + 63) / 64;
          const int nmb = (g.nmon + 63) / 64, nbx = (int)(g.ld / 64);
          bf16x8* a3 = (bf16x8*)(w + L.dl_split);
          bf16x8* v3 = a3 + (size_t)kSplitUnits * g.R;
          const int T = nb * (nb + 1) / 2 + nmb * nbx;
          const unsigned gx = (unsigned)((nx + 255) / 256);
          auto run = [&](auto kc) {
            constexpr int KC = decltype(kc)::value;
            // two workgroups per compute unit up to 64 terms, one (one wave per SIMD,
            // the 128 terms' A parts in 192 registers) beyond
            const int P = band_workgroups(KC == 8 ? 1 : 2);
            hipLaunchKernelGGL(k_flush_pack_s3<KC>, dim3(gx, 2 * KC), blk, 0, s, g.R, g.ld, count, cu, vv,
                               a3, v3);
            hipLaunchKernelGGL(k_flush_c64_s3<KC>, dim3((unsigned)P), blk, 0, s, g.N, g.R, g.ld, count,
                               (const bf16x8*)a3, (const bf16x8*)v3, G, nb, (T + P - 1) / P, g.packed,
                               g.mon_base, sw);
          };
          if (bound <= 32) run(std::integral_constant<int, 2>{});
          else if (bound <= 64) run(std::integral_constant<int, 4>{});
          else run(std::integral_constant<int, 8>{});
          monitors_done = true;
          break;
        }
        // upper triangle only, pair-interleaved terms in the unused halves of
        // the term buffers (complex64 slots take 8 of their 16 bytes)
        const int nb = (g.N + 63) / 64;
        f32x4* cu2 = (f32x4*)(w + L.dl_CUs + (size_t)GFO_MAX_DELAY * g.R * 8);
        f32x4* vv2 = (f32x4*)(w + L.dl_Vs + (size_t)GFO_MAX_DELAY * g.ld * 8);
        hipLaunchKernelGGL(k_flush_pack, dim3((unsigned)((nx + 255) / 256), GFO_MAX_DELAY / 2), blk, 0, s,
                           g.R, g.ld, count, cu, vv, cu2, vv2);
        // the triangle's tiles, then the monitor rows' (no separate monitor kernel)
        const int nmb = (g.nmon + 63) / 64, nbx = (int)(g.ld / 64);
        unsigned ntiles = (unsigned)(nb * (nb + 1) / 2 + nmb * nbx);
        // the XCD tile order keeps every operand re-read in the XCD's L2 (at 128
        // terms: 1.05x the minimal HBM traffic instead of 1.8x, 2 % slower); the
        // band form in column segments does for 33 to 64 terms
        const bool xord = fv == 2 || fv >= 4;
        // the band form addresses a 64-row G tile with 32-bit byte offsets
        const bool band = (fv == 3 || fv == 4) && g.ld * 64 * 8 < ((int64_t)1 << 31);
        if (xord) {
          int mx = 0;
          for (int x = 0; x < 8; ++x) {
            const int c = xcd_tile_count(nb, nbx, nmb, x);
            mx = c > mx ? c : mx;
          }
          ntiles = 8u * (unsigned)mx;
        }
        const dim3 tri(ntiles);
        monitors_done = true;
        const f32x4* c2 = (const f32x4*)cu2;
        const f32x4* v2 = (const f32x4*)vv2;
        if (bound <= 16) {
          if (xord) hipLaunchKernelGGL((k_flush_c64_pair<4, 4, true>), tri, blk, 0, s, g.N, g.R, g.ld, count, c2, v2, G, nb, g.packed, g.mon_base);
          else hipLaunchKernelGGL((k_flush_c64_pair<4, 4>), tri, blk, 0, s, g.N, g.R, g.ld, count, c2, v2, G, nb, g.packed, g.mon_base);
        } else if (bound <= 32) {
          if (xord) hipLaunchKernelGGL((k_flush_c64_pair<4, 8, true>), tri, blk, 0, s, g.N, g.R, g.ld, count, c2, v2, G, nb, g.packed, g.mon_base);
          else hipLaunchKernelGGL((k_flush_c64_pair<4, 8>), tri, blk, 0, s, g.N, g.R, g.ld, count, c2, v2, G, nb, g.packed, g.mon_base);
        } else if (bound <= 64) {
          if (band) {
            const int P = band_workgroups();
            const int T = nb * (nb + 1) / 2 + nmb * nbx;
            if (fv == 4)
              hipLaunchKernelGGL((k_flush_c64_band<16, true>), dim3((unsigned)P), blk, 0, s, g.N, g.R, g.ld, count, c2,
                                 v2, G, nb, (T + P - 1) / P, g.packed, g.mon_base);
            else
              hipLaunchKernelGGL((k_flush_c64_band<16, false>), dim3((unsigned)P), blk, 0, s, g.N, g.R, g.ld, count, c2,
                                 v2, G, nb, (T + P - 1) / P, g.packed, g.mon_base);
          } else if (xord) {
            hipLaunchKernelGGL((k_flush_c64_pair<4, 16, true>), tri, blk, 0, s, g.N, g.R, g.ld, count, c2, v2, G, nb, g.packed, g.mon_base);
          } else {
            hipLaunchKernelGGL((k_flush_c64_pair<4, 16>), tri, blk, 0, s, g.N, g.R, g.ld, count, c2, v2, G, nb, g.packed, g.mon_base);
          }
        } else {
          if (xord) hipLaunchKernelGGL((k_flush_c64_pair<4, 32, true>), tri, blk, 0, s, g.N, g.R, g.ld, count, c2, v2, G, nb, g.packed, g.mon_base);
          else hipLaunchKernelGGL((k_flush_c64_pair<4, 32>), tri, blk, 0, s, g.N, g.R, g.ld, count, c2, v2, G, nb, g.packed, g.mon_base);
        }
        st->lower_stale = 1;
        break;
      }
    }
    e = hipGetLastError();
    if (e != hipSuccess) return note_hip(e);
    // the timed interval is the design-block kernel alone
    if (hipError_t er = record_event(after, s)) return note_hip(er);
    // the monitor rows (the FOM monitor's terms are stored as zeros)
    if (!monitors_done) {
      hipLaunchKernelGGL((k_flush_c64_tm<1, true>),
                         dim3((unsigned)((g.N + 63) / 64), (unsigned)((g.nmon + 63) / 64)), blk, 0, s,
                         g.R, g.R, g.ld, count, cu, vv, G, g.N);
      e = note_hip(hipGetLastError());
    }
  } else {
    if (hipError_t er = record_event(before, s)) return note_hip(er);
    e = launch_zgemm_update_f64(g, count, (const double2*)(w + L.dl_CUs),
                                (const double2*)(w + L.dl_Vs), (double2*)st->G, s);
    if (e == hipSuccess) e = record_event(after, s);
    if (e != hipSuccess) return note_hip(e);
    st->lower_stale = 1;
  }
  if (e != hipSuccess) return e;
  return launch_dl_reset(g, st, L, s);
}

// Upper triangle of the design block copied into its strict lower triangle:
// workgroup t takes 32 x 32 tile (by, bx) on or above the diagonal (tri_tile
// order), reads it row by row into LDS and writes its transpose into tile
// (bx, by) row by row (on diagonal tiles only below the diagonal).
template <typename T>
__global__ __launch_bounds__(256) void k_sync_lower(int N, int64_t ld, T* __restrict__ G, int nb) {
  __shared__ T tile[32][33];
  int by, bx;
  tri_tile((int)blockIdx.x, nb, by, bx);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = by * 32 + ty + 8 * k, c = bx * 32 + tx;
    if (r < N && c < N) tile[ty + 8 * k][tx] = G[(int64_t)r * ld + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int lr = ty + 8 * k, row = bx * 32 + lr, col = by * 32 + tx;
    if (row < N && col < N && (bx != by || lr > tx)) G[(int64_t)row * ld + col] = tile[tx][lr];
  }
}

hipError_t launch_sync_lower(const Geo& g, gfo_state* st, hipStream_t s) {
  const int nb = (g.N + 31) / 32;
  const dim3 grid((unsigned)((int64_t)nb * (nb + 1) / 2));
  if (g.dtype == GFO_C64)
    hipLaunchKernelGGL(k_sync_lower<float2>, grid, dim3(256), 0, s, g.N, g.ld, (float2*)st->G, nb);
  else
    hipLaunchKernelGGL(k_sync_lower<double2>, grid, dim3(256), 0, s, g.N, g.ld, (double2*)st->G, nb);
  return note_hip(hipGetLastError());
}

}  // namespace gfo
