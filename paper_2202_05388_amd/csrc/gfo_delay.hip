// Deferred rank-1 updates.  Eq. form10 applied move by move gives
//   G_t = G_base + sum_{s < t} cu_s v_s^T,   cu_s = c_s G_s[:, j_s],  v_s = G_s[j_s, :],
// so the design block (and the monitor rows other than the FOM monitor's) can be
// brought up to date later, in one rank-r product (gfo_flush.hip), while
// everything the scores read (E, diag64, the FOM monitor row) is updated at
// once.  Column j and row j of the current matrix are the base entries plus the
// pending terms.
#include "gfo_internal.hpp"

namespace gfo {

// Pending terms are stored slot-major, CUs[s * R + r] and Vs[s * ld + q]: the
// consecutive elements of one term are contiguous, which both the per-move
// gathers (one element per lane, all terms of it) and the flush read coalesced.

// x + a b in FP64, rounded to the storage type: the E, monitor-row and (via
// emon) monitor-field updates of every path go through this one expression.
template <typename T>
__device__ __forceinline__ T axpy_st(T x, T a, double2 b) {
  return St<T>::from_d(cadd(St<T>::to_d(x), cmul(St<T>::to_d(a), b)));
}

// The move's scalars, from the pick and the values at its pixel that no thread
// of this launch writes (eps_idx[j], diag64[j], E[j], the term count); cur, dj
// and Ej are read at jc, the pick's pixel clamped into range.
template <typename T>
__device__ __forceinline__ Snap deferred_snapshot(const Geo& g, const gfo_pick pk, int cur,
                                                  double2 dj, T Ej, int cnt) {
  Snap s = {};
  s.j = -1;
  const int j = pk.pixel, e = pk.eps_idx;
  if (j >= 0 && j < g.N && e >= 0 && e < g.n_eps && e != cur) {
    const double a = g.k0sq * (g.eps[e] - g.eps[cur]);
    const double2 den = make_double2(1.0 - a * dj.x, -a * dj.y);
    if (cabs2(den) < 1e-24) {
      s.pad1 = 1;                           // singular: refused, flagged by the next kernel
    } else {
      s.j = j;
      s.e_new = e;
      s.alpha = a;
      s.c = rdiv(a, den);
      s.Ej = St<T>::to_d(Ej);
      s.dj = dj;
      s.slot = cnt;
    }
  }
  return s;
}

// Column j and row j of the current matrix G_t = G_base + sum_s cu_s v_s^T:
//   row entries    v_q = G[j, q] + sum_s CU_s[j] V_s[q]  for q < N (0 beyond);
//   design column  u_i = v_i: the design block is symmetric (reciprocity), and
//                  so is each pending term restricted to it;
//   monitor rows   u_{N+m} = G[N+m, j] + sum_s CU_s[N+m] V_s[j], except the FOM
//                  monitor's row, which is current.
// cu = c u and v are stored as term `slot` (the FOM monitor's entry as zero: its
// row already has the term) and in cu_out / v_out; the monitor rows also give E
// at the monitors after the move, emon[m] = E[N+m] + cu[N+m] E_j.  Workgroup 0
// publishes the snapshot for the next kernel.  Nothing written here is read by
// this launch.
//
// Elements e of [0, mpad + ld), mpad = nmon rounded up to kGatherElems: monitor
// row N + e for e < nmon (none for nmon <= e < mpad), else row entry
// q = e - mpad, so that a workgroup holds one kind only.  A workgroup of
// kGatherParts waves takes kGatherElems consecutive elements, one per lane;
// wave w sums the terms
// [w B, (w + 1) B) from zero in slot order, the partial
// sums meet in LDS, and wave 0 adds them pairwise to the base entry and stores.
// Two phases, so that the loads that do not depend on the pick are in flight
// while it is taken: gather_prefetch reads the term count and the lane's own
// operand of each of its wave's terms (CU_s[N+m] or V_s[q], through buffer
// loads whose range ends at the term count, so that slots past it read as zero
// without a branch); gather_finish
// issues the loads that depend on the pick at once (the pixel's scalars, the
// base entries, and the terms' entries at j, staged once per workgroup in LDS).
// B terms per wave: 16 while the state's delay is at most 64, else 32 (the
// slots of a term buffer of 4 B); every path of a state uses the same B, so
// their sums agree bit for bit.
constexpr int kGatherParts = 4;
constexpr int kGatherElems = 64;
static_assert(kGatherParts * 64 == 256, "one wave per part");
static_assert(GFO_MAX_DELAY <= kGatherParts * 32, "two term batches cover every delay");

__host__ __device__ constexpr int gather_batch(int delay) { return delay <= 64 ? 16 : 32; }

template <typename T, int B>
struct GatherPre {
  int cnt;                    // pending terms = this move's slot
  T a[B];                     // the lane's operands of its wave's terms
};

__host__ __device__ inline int gather_mpad(const Geo& g) {
  return (g.nmon + kGatherElems - 1) / kGatherElems * kGatherElems;
}

// The element of this lane: e, whether it is a monitor row (uniform over the
// workgroup), and whether it exists.
struct GatherElem {
  int64_t e;
  bool mon, live;
  int64_t i, q;               // monitor row N + e, or row entry q (clamped)
};

__device__ __forceinline__ GatherElem gather_elem(const Geo& g) {
  GatherElem el;
  const int mpad = gather_mpad(g);
  el.e = (int64_t)blockIdx.x * kGatherElems + (threadIdx.x & 63);
  el.mon = (int64_t)blockIdx.x * kGatherElems < mpad;
  el.live = el.mon ? el.e < g.nmon : el.e - mpad < g.ld;
  el.i = el.mon ? g.N + (el.live ? el.e : 0) : 0;
  el.q = el.mon ? 0 : (el.live ? el.e - mpad : 0);
  return el;
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ float2 buf_load<float2>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double2 buf_load<double2>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

template <typename T, int B>
__device__ __forceinline__ void gather_prefetch_n(const Geo& g, int cnt, const T* __restrict__ CUs,
                                                  const T* __restrict__ Vs, GatherPre<T, B>& pre) {
  pre.cnt = cnt;
  const GatherElem el = gather_elem(g);
  // one resource per workgroup: its range ends at the term count
  const int64_t stride = el.mon ? g.R : g.ld;
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(el.mon ? CUs : Vs), (short)0, (int)(pre.cnt * stride * (int64_t)sizeof(T)), 0x00020000);
  const unsigned off = (unsigned)((el.mon ? el.i : el.q) * (int64_t)sizeof(T));
  const int s0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * B;
#pragma unroll
  for (int k = 0; k < B; ++k)
    pre.a[k] = buf_load<T>(r, off + (unsigned)((s0 + k) * stride * (int64_t)sizeof(T)));
}

template <typename T, int B>
__device__ __forceinline__ void gather_prefetch(const Geo& g, const int32_t* __restrict__ count,
                                                const T* __restrict__ CUs,
                                                const T* __restrict__ Vs, GatherPre<T, B>& pre) {
  gather_prefetch_n<T, B>(g, __builtin_amdgcn_readfirstlane(*count), CUs, Vs, pre);
}

template <typename T, int B>
__device__ __forceinline__ void gather_finish(const Geo& g, const gfo_pick pk,
                                              const GatherPre<T, B>& pre, const T* __restrict__ G,
                                              const T* __restrict__ E,
                                              const double2* __restrict__ diag64,
                                              const uint8_t* __restrict__ eps_idx,
                                              Snap* __restrict__ snap_out, T* __restrict__ CUs,
                                              T* __restrict__ Vs, T* __restrict__ cu_out,
                                              T* __restrict__ v_out, T* __restrict__ emon) {
  __shared__ T yj[2][GFO_MAX_DELAY];              // V_s[j] (monitor rows), CU_s[j] (row entries)
  __shared__ double2 part[kGatherParts - 1][kGatherElems];
  const int cnt = pre.cnt;
  const int jc = __builtin_amdgcn_readfirstlane(pk.pixel >= 0 && pk.pixel < g.N ? pk.pixel : 0);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const GatherElem el = gather_elem(g);
  const int64_t e = el.e, i = el.i, q = el.q;
  const bool mon = el.mon, live = el.live;
  // every load that depends on the pick, issued together
  const int cur = eps_idx[jc];
  const double2 dj = diag64[jc];
  const T Ej = E[jc];
  T base = St<T>::from_d(make_double2(0.0, 0.0));
  if (w == 0) base = mon ? G[g_off(g, i, jc)] : G[g_at(g, jc, q)];
  if (threadIdx.x < cnt) yj[0][threadIdx.x] = Vs[(int64_t)threadIdx.x * g.ld + jc];
  if (threadIdx.x >= 64 && threadIdx.x - 64 < cnt)
    yj[1][threadIdx.x - 64] = CUs[(int64_t)(threadIdx.x - 64) * g.R + jc];
  const Snap sn = deferred_snapshot<T>(g, pk, cur, dj, Ej, cnt);
  if (blockIdx.x == 0 && threadIdx.x == 0) *snap_out = sn;
  const int j = __builtin_amdgcn_readfirstlane(sn.j);
  __syncthreads();
  // the terms of an entry: design row entries other than the pivot, and the
  // monitor rows except the FOM monitor's
  const bool terms = mon ? (e != g.m0) : (q < g.N && q != j);
  const int s0 = w * B;
  double2 acc = make_double2(0.0, 0.0);
  if (j >= 0 && terms) {
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (s0 + k < cnt) acc = cadd(acc, cmul(St<T>::to_d(pre.a[k]), St<T>::to_d(yj[mon ? 0 : 1][s0 + k])));
  }
  if (w > 0) part[w - 1][lane] = acc;
  __syncthreads();
  if (j < 0 || w != 0 || !live) return;
  acc = cadd(cadd(acc, part[0][lane]), cadd(part[1][lane], part[2][lane]));
  const int slot = cnt;
  if (mon) {
    const double2 u = e != g.m0 ? cadd(St<T>::to_d(base), acc) : St<T>::to_d(base);
    const T cu = St<T>::from_d(cmul(sn.c, u));
    CUs[(int64_t)slot * g.R + i] = e != g.m0 ? cu : St<T>::from_d(make_double2(0.0, 0.0));
    cu_out[i] = cu;
    emon[e] = axpy_st<T>(E[i], cu, sn.Ej);
  } else {
    double2 v = make_double2(0.0, 0.0);
    if (q < g.N) v = q == j ? sn.dj : cadd(St<T>::to_d(base), acc);
    const T vv = St<T>::from_d(v);
    Vs[(int64_t)slot * g.ld + q] = vv;
    v_out[q] = vv;
    if (q < g.N) {
      const T cu = St<T>::from_d(cmul(sn.c, v));
      CUs[(int64_t)slot * g.R + q] = cu;
      cu_out[q] = cu;
    }
  }
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_gather_dl(
    Geo g, const gfo_pick* __restrict__ pick, const T* __restrict__ G, const T* __restrict__ E,
    const double2* __restrict__ diag64, const uint8_t* __restrict__ eps_idx,
    const int32_t* __restrict__ count, Snap* __restrict__ snap_out, T* __restrict__ CUs,
    T* __restrict__ Vs, T* __restrict__ cu_out, T* __restrict__ v_out, T* __restrict__ emon) {
  GatherPre<T, B> pre;
  gather_prefetch<T, B>(g, count, CUs, Vs, pre);
  gather_finish<T, B>(g, *pick, pre, G, E, diag64, eps_idx, snap_out, CUs, Vs, cu_out, v_out, emon);
}

// Fused pick + gather: every wave takes the greedy pick from the score
// summaries (identical in all of them: the same reads, exact max and min
// reductions) while its pick-independent gather loads are in flight; workgroup
// 0 records the pick in `pick_out`.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_select_gather(
    Geo g, const double* __restrict__ scores, const double* __restrict__ partial,
    const int* __restrict__ pfirst, int nblk, double tau, gfo_pick* __restrict__ pick_out,
    const T* __restrict__ G, const T* __restrict__ E, const double2* __restrict__ diag64,
    const uint8_t* __restrict__ eps_idx, const int32_t* __restrict__ count,
    Snap* __restrict__ snap_out, T* __restrict__ CUs, T* __restrict__ Vs, T* __restrict__ cu_out,
    T* __restrict__ v_out, T* __restrict__ emon) {
  // the summaries first: waiting for them then does not wait for the term
  // operands (vector loads complete in issue order)
  PickPre<> pp;
  pick_wave_load(partial, pfirst, nblk, pp);
  const double fom = cabs2(St<T>::to_d(E[g.N + g.m0]));
  __builtin_amdgcn_sched_barrier(0);
  GatherPre<T, B> pre;
  gather_prefetch<T, B>(g, count, CUs, Vs, pre);
  __builtin_amdgcn_sched_barrier(0);
  gfo_pick pk = pick_wave_take(g, fom, pp, scores, tau, false);
  gather_finish<T, B>(g, pk, pre, G, E, diag64, eps_idx, snap_out, CUs, Vs, cu_out, v_out, emon);
  // the record of the pick, off the gather's critical path
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (pk.pixel >= 0) {
      pk.fom_new = scores[pk.pixel * g.n_eps + pk.eps_idx];
      pk.dfom = pk.fom_new - fom;
    }
    *pick_out = pk;
  }
}

// The move's elementwise part for one index q (design pixel or monitor row):
// E_q += cu_q E_j (the monitor fields are taken from emon, computed by the
// gather with the same expression), diag64 (q != j: += cu_q v_q; q = j:
// d_j / (1 - alpha d_j)) and eps_idx[j]; the FOM monitor row G[N+m0, q] +=
// cu[N+m0] v_q (the scores read it; the other monitor rows take their pending
// terms at the flush, like the design block).  Shared by the per-call path and
// the fused greedy loop.
template <typename T>
__device__ __forceinline__ void elementwise_move(const Geo& g, const Snap& sn, int64_t q,
                                                 const T* __restrict__ cu,
                                                 const T* __restrict__ v,
                                                 const T* __restrict__ emon, T* __restrict__ G,
                                                 T* __restrict__ E, double2* __restrict__ diag64,
                                                 uint8_t* __restrict__ eps_idx) {
  const int j = sn.j;
  {
    if (q < g.N) {
      E[q] = axpy_st<T>(E[q], cu[q], sn.Ej);
      if (q == j) {
        const double2 d = sn.dj;
        diag64[j] = cmul(d, rdiv(1.0, make_double2(1.0 - sn.alpha * d.x, -sn.alpha * d.y)));
        eps_idx[j] = (uint8_t)sn.e_new;
      } else {
        diag64[q] = cadd(diag64[q], cmul(St<T>::to_d(cu[q]), St<T>::to_d(v[q])));
      }
    } else if (q < g.R) {
      E[q] = emon[q - g.N];
    }
  }
  if (q >= g.ld) return;
  T* p = G + g_off(g, g.N + g.m0, q);
  *p = axpy_st<T>(*p, cu[g.N + g.m0], St<T>::to_d(v[q]));
}

// Bookkeeping of an applied move (history, move counter, pending-term count).
__device__ __forceinline__ void record_move(const Snap& sn, int32_t* __restrict__ flips,
                                            int flip_cap, int32_t* __restrict__ n_flips,
                                            int32_t* __restrict__ status,
                                            int32_t* __restrict__ count) {
  const int n = *n_flips;
  if (n < flip_cap) {
    flips[2 * n] = sn.j;
    flips[2 * n + 1] = sn.e_new;
  } else {
    atomicOr(status, GFO_STATUS_HISTORY_FULL);
  }
  *n_flips = n + 1;
  *count = sn.slot + 1;
}

// Applies the move's elementwise part.  Grid x covers max(R, ld).
template <typename T>
__global__ void k_mon_dl(Geo g, const Snap* __restrict__ snap, const T* __restrict__ cu,
                         const T* __restrict__ v, const T* __restrict__ emon, T* __restrict__ G,
                         T* __restrict__ E, double2* __restrict__ diag64,
                         uint8_t* __restrict__ eps_idx, int32_t* __restrict__ flips, int flip_cap,
                         int32_t* __restrict__ n_flips, int32_t* __restrict__ status,
                         int32_t* __restrict__ count) {
  const Snap sn = *snap;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sn.j < 0) {
    if (q == 0 && sn.pad1) atomicOr(status, GFO_STATUS_SINGULAR);
    return;
  }
  if (q == 0) record_move(sn, flips, flip_cap, n_flips, status, count);
  elementwise_move<T>(g, sn, q, cu, v, emon, G, E, diag64, eps_idx);
}

// Fused greedy loop, first kernel of a move.  Grid x covers max(R, ld) indices
// q: the previous move's elementwise part for index q (if apply_prev) and then
// the scores of pixel q (workgroup b covers pixels [256 b, 256 b + 256) and
// writes partial[b] for b < nblk).  Thread q updates exactly the values it then
// scores with (E_q, diag64[q], eps_idx[q], G[N+m0, q]) and scores from
// registers; E at the FOM monitor comes from emon.
// The expressions are those of k_mon_dl and k_score, so the state and the scores
// are bit for bit those of the per-call path.
template <typename T>
__device__ __forceinline__ void mon_score_body(
    const Geo& g, int apply_prev, const Snap* __restrict__ snap, const T* __restrict__ cu,
    const T* __restrict__ v, const T* __restrict__ emon, T* __restrict__ G, T* __restrict__ E,
    double2* __restrict__ diag64, uint8_t* __restrict__ eps_idx, int32_t* __restrict__ flips,
    int flip_cap, int32_t* __restrict__ n_flips, int32_t* __restrict__ status,
    int32_t* __restrict__ count, uint32_t mask, double tau, double* __restrict__ scores,
    double* __restrict__ partial, int* __restrict__ pfirst, int nblk) {
  __shared__ double sh[kScoreThreads / 64];
  __shared__ int shi[kScoreThreads / 64];
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // every load of this thread first and unconditionally (indices clamped to
  // valid elements; values past the ends are not used), together with the
  // move's snapshot, so that the kernel waits for memory once before its stores
  const int64_t qc = q < g.N ? q : g.N - 1, ql = q < g.ld ? q : g.ld - 1;
  const int64_t qm = q < g.N ? 0 : (q - g.N < g.nmon ? q - g.N : g.nmon - 1);
  T Eq = E[qc];
  double2 dq = diag64[qc];
  int cur = eps_idx[qc];
  const T cuq = cu[qc], vq = v[ql], emq = emon[qm];
  T* __restrict__ grow = G + g_off(g, g.N + g.m0, 0);
  T grow_q = grow[ql];
  const T em0 = emon[g.m0], e0 = E[g.N + g.m0], cum0 = cu[g.N + g.m0];
  __builtin_amdgcn_sched_barrier(0);
  Snap sn;
  sn.j = -1;
  if (apply_prev) sn = *snap;
  const bool moved = sn.j >= 0;
  const double2 Em0 = St<T>::to_d(moved ? em0 : e0);
  if (moved) {
    grow_q = axpy_st<T>(grow_q, cum0, St<T>::to_d(vq));
    if (q < g.ld) grow[q] = grow_q;
  }
  double best = -INFINITY;
  bool bad = false;
  double F[GFO_MAX_EPS];
  if (q < g.N) {
    if (moved) {
      Eq = axpy_st<T>(Eq, cuq, sn.Ej);
      E[q] = Eq;
      if (q == sn.j) {
        const double2 dd = sn.dj;
        dq = cmul(dd, rdiv(1.0, make_double2(1.0 - sn.alpha * dd.x, -sn.alpha * dd.y)));
        cur = sn.e_new;
        eps_idx[q] = (uint8_t)cur;
      } else {
        dq = cadd(dq, cmul(St<T>::to_d(cuq), St<T>::to_d(vq)));
      }
      diag64[q] = dq;
    }
    const double2 gE = cmul(St<T>::to_d(grow_q), St<T>::to_d(Eq));
    best = score_pixel(g, (int)q, cur, dq, gE, Em0, mask, scores, &bad, F);
  } else if (moved && q < g.R) {
    E[q] = emq;
  }
  score_block_end(g, best, (int)(q < g.N ? q : g.N), true, F, tau, partial, pfirst, nblk, sh, shi);
  if (bad) atomicOr(status, GFO_STATUS_NONFINITE);
  // the move's bookkeeping (nothing in this launch reads it)
  if (!moved && apply_prev && q == 0 && sn.pad1) atomicOr(status, GFO_STATUS_SINGULAR);
  if (moved && q == 0) record_move(sn, flips, flip_cap, n_flips, status, count);
}

template <typename T>
__global__ __launch_bounds__(kScoreThreads) void k_mon_score(
    Geo g, int apply_prev, const Snap* __restrict__ snap, const T* __restrict__ cu,
    const T* __restrict__ v, const T* __restrict__ emon, T* __restrict__ G, T* __restrict__ E,
    double2* __restrict__ diag64, uint8_t* __restrict__ eps_idx, int32_t* __restrict__ flips,
    int flip_cap, int32_t* __restrict__ n_flips, int32_t* __restrict__ status,
    int32_t* __restrict__ count, uint32_t mask, double tau, double* __restrict__ scores,
    double* __restrict__ partial, int* __restrict__ pfirst, int nblk) {
  mon_score_body<T>(g, apply_prev, snap, cu, v, emon, G, E, diag64, eps_idx, flips, flip_cap,
                    n_flips, status, count, mask, tau, scores, partial, pfirst, nblk);
}

__global__ void k_dl_reset(int32_t* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count = 0;
}

hipError_t launch_dl_reset(const Geo&, gfo_state* st, const Layout& L, hipStream_t s) {
  hipLaunchKernelGGL(k_dl_reset, dim3(1), dim3(64), 0, s, (int32_t*)((char*)st->work + L.dl_hdr));
  return note_hip(hipGetLastError());
}

// One kernel per move (fused greedy loop, deferred mode, when the pixels fit
// kScoreMaxBlocks summaries of kGatherElems).  Kernel t takes the pick of move t
// from the summaries the previous kernel left, gathers row j and the monitor
// rows of column j as k_select_gather does, then each row-entry lane applies
// the move's elementwise part to its own pixel (E, FP64 diagonal, material,
// FOM monitor row) and scores that pixel for move t + 1; wave 0 of each
// workgroup leaves one summary per kGatherElems pixels.  Nothing is written
// during a kernel that another workgroup of it reads: the pivot's values
// (E[j], diag64[j], eps_idx[j], G[N+m0, j]) after the move travel in the
// move's snapshot and reach memory in the next kernel, or in k_move_finish
// (after the last move of a call and before a flush: the flush rewrites the
// FOM monitor row, so it must see the pivot's entry); the fields at the
// monitors go through emon buffers, and E[N+m] is written one kernel late; the
// term count is carried by the snapshots (the first kernel of a call, and the
// flush, read it from memory, which k_move_finish brings up to date);
// snapshots, scores and summaries alternate between two sets of buffers.  The expressions are those of the per-call path (k_gather_dl,
// k_mon_dl, k_score), so the state and the picks are bit for bit the same.
template <typename T, int PPL, int B>
__device__ __forceinline__ void move_body(
    const Geo& g, int has_prev, int flushed, const Snap* __restrict__ snap_prev,
    Snap* __restrict__ snap_out, const double* __restrict__ scores_prev,
    const double* __restrict__ partial_prev, const int* __restrict__ pfirst_prev, int nblk_prev,
    int bpix_prev, double* __restrict__ scores_next, double* __restrict__ partial_next,
    int* __restrict__ pfirst_next, const T* __restrict__ emon_prev, T* __restrict__ emon_next,
    uint32_t mask, double tau, gfo_pick* __restrict__ pick_out, T* __restrict__ G,
    T* __restrict__ E, double2* __restrict__ diag64, uint8_t* __restrict__ eps_idx,
    const int32_t* __restrict__ count, int32_t* __restrict__ flips, int flip_cap,
    int32_t* __restrict__ n_flips, int32_t* __restrict__ status, T* __restrict__ CUs,
    T* __restrict__ Vs) {
  __shared__ T yj[2][GFO_MAX_DELAY];              // V_s[j] (monitor rows), CU_s[j] (row entries)
  __shared__ double2 part[kGatherParts - 1][kGatherElems];
  const T zero = St<T>::from_d(make_double2(0.0, 0.0));
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const GatherElem el = gather_elem(g);
  const int64_t e = el.e, i = el.i, q = el.q;
  const bool mon = el.mon, live = el.live;
  T* __restrict__ grow = G + g_off(g, g.N + g.m0, 0);
  // loads that need nothing else: the summaries first, then the lane's operand
  // of every slot of its wave's terms (those past the term count, not known
  // yet, are not used), then this lane's own values (its pixel, or its
  // monitor's field)
  PickPre<PPL> pp;
  pick_wave_load(partial_prev, pfirst_prev, nblk_prev, pp);
  GatherPre<T, B> pre;
  gather_prefetch_n<T, B>(g, kGatherParts * B, CUs, Vs, pre);
  const int64_t qc = q < g.N ? q : g.N - 1;
  const T Eown = E[mon ? i : qc];
  const double2 dq = diag64[qc];
  const int curq = eps_idx[qc];
  const T gq = grow[qc];
  const T emon_e = has_prev && mon ? emon_prev[live ? e : 0] : Eown;
  const T em0_prev = has_prev ? emon_prev[g.m0] : E[g.N + g.m0];
  __builtin_amdgcn_sched_barrier(0);
  Snap sp;
  sp.j = -1;
  sp.cnt_after = 0;
  if (has_prev) sp = *snap_prev;
  // after a flush the previous move's values are in memory (k_move_finish ran
  // before it, so that the flush saw them)
  const bool carry = has_prev && !flushed;
  const int cnt = flushed ? 0 : (has_prev ? sp.cnt_after : *count);
  const double fom = cabs2(St<T>::to_d(em0_prev));
  const gfo_pick pk = pick_wave_take(g, fom, pp, scores_prev, tau, false, bpix_prev);
  const int jc = __builtin_amdgcn_readfirstlane(pk.pixel >= 0 && pk.pixel < g.N ? pk.pixel : 0);
  // the pivot's values before this move (the previous pivot's from its snapshot)
  const bool ovr = carry && sp.j >= 0 && sp.j == jc;
  int cur = eps_idx[jc];
  double2 dj = diag64[jc];
  T Ej = E[jc], gm0j = grow[jc];
  if (ovr) {
    cur = sp.e_new;
    dj = sp.dj_new;
    Ej = St<T>::from_d(sp.Ej_new);
    gm0j = St<T>::from_d(sp.gm0_new);
  }
  T base = zero;
  if (w == 0) base = mon ? (e == g.m0 ? gm0j : G[g_off(g, i, jc)]) : G[g_at(g, jc, q)];
  if (threadIdx.x < cnt) yj[0][threadIdx.x] = Vs[(int64_t)threadIdx.x * g.ld + jc];
  if (threadIdx.x >= 64 && threadIdx.x - 64 < cnt)
    yj[1][threadIdx.x - 64] = CUs[(int64_t)(threadIdx.x - 64) * g.R + jc];
  const Snap sn = deferred_snapshot<T>(g, pk, cur, dj, Ej, cnt);
  const int j = __builtin_amdgcn_readfirstlane(sn.j);
  const bool moved = j >= 0;
  // the FOM monitor's term entry and field after the move, alike everywhere
  const T cu_m0 = moved ? St<T>::from_d(cmul(sn.c, St<T>::to_d(gm0j))) : zero;
  const T em0_new = moved ? axpy_st<T>(em0_prev, cu_m0, sn.Ej) : em0_prev;
  __syncthreads();
  const bool terms = moved && (mon ? e != g.m0 : (q < g.N && q != j));
  const int s0 = w * B;
  double2 acc = make_double2(0.0, 0.0);
  if (terms) {
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (s0 + k < cnt) acc = cadd(acc, cmul(St<T>::to_d(pre.a[k]), St<T>::to_d(yj[mon ? 0 : 1][s0 + k])));
  }
  if (w > 0) part[w - 1][lane] = acc;
  __syncthreads();
  if (w != 0) return;
  acc = cadd(cadd(acc, part[0][lane]), cadd(part[1][lane], part[2][lane]));
  const int slot = cnt;
  double best = -INFINITY;
  double F[GFO_MAX_EPS];
  bool bad = false;
  if (mon) {
    if (live) {
      if (has_prev) E[i] = emon_e;                // the previous move's field (no reader here)
      T em = emon_e;
      if (moved) {
        const double2 u = e != g.m0 ? cadd(St<T>::to_d(base), acc) : St<T>::to_d(base);
        const T cu = St<T>::from_d(cmul(sn.c, u));
        CUs[(int64_t)slot * g.R + i] = e != g.m0 ? cu : zero;
        em = axpy_st<T>(em, cu, sn.Ej);
      }
      emon_next[e] = em;
    }
  } else if (live) {
    T vv = zero, cuq = zero;
    if (moved) {
      double2 v = make_double2(0.0, 0.0);
      if (q < g.N) v = q == j ? sn.dj : cadd(St<T>::to_d(base), acc);
      vv = St<T>::from_d(v);
      Vs[(int64_t)slot * g.ld + q] = vv;
      if (q < g.N) {
        cuq = St<T>::from_d(cmul(sn.c, v));
        CUs[(int64_t)slot * g.R + q] = cuq;
      }
    }
    if (q < g.N) {
      // pixel q before this move (the previous pivot's values from its snapshot)
      const bool prevp = carry && sp.j >= 0 && q == sp.j;
      T Ec = prevp ? St<T>::from_d(sp.Ej_new) : Eown;
      double2 dc = prevp ? sp.dj_new : dq;
      int cc = prevp ? sp.e_new : curq;
      T gc = prevp ? St<T>::from_d(sp.gm0_new) : gq;
      if (moved) {
        Ec = axpy_st<T>(Ec, cuq, sn.Ej);
        if (q == j) {
          dc = cmul(sn.dj, rdiv(1.0, make_double2(1.0 - sn.alpha * sn.dj.x, -sn.alpha * sn.dj.y)));
          cc = sn.e_new;
        } else {
          dc = cadd(dc, cmul(St<T>::to_d(cuq), St<T>::to_d(vv)));
        }
        gc = axpy_st<T>(gc, cu_m0, St<T>::to_d(vv));
      }
      if ((moved || prevp) && !(moved && q == j)) {
        E[q] = Ec;
        diag64[q] = dc;
        eps_idx[q] = (uint8_t)cc;
        grow[q] = gc;
      }
      const double2 gE = cmul(St<T>::to_d(gc), St<T>::to_d(Ec));
      best = score_pixel(g, (int)q, cc, dc, gE, St<T>::to_d(em0_new), mask, scores_next, &bad, F);
    }
  }
  if (!mon) {
    // this workgroup's pixels: its best score and the lowest index within the
    // tie band of that best
    const double bb = wave_max(best);
    int f = 0x7fffffff;
    if (live && q < g.N && bb > -INFINITY) f = first_at_least(g, (int)q, F, tie_threshold(bb, tau));
    f = wave_min(f);
    const int64_t pb = (int64_t)blockIdx.x - gather_mpad(g) / kGatherElems;
    if (lane == 0 && pb * kGatherElems < g.N) {
      partial_next[pb] = bb;
      pfirst_next[pb] = f;
    }
  }
  if (bad) atomicOr(status, GFO_STATUS_NONFINITE);
  if (blockIdx.x == 0 && lane == 0) {
    *snap_out = sn;
    snap_out->cnt_after = moved ? cnt + 1 : cnt;
    if (moved) {
      const T cuj = St<T>::from_d(cmul(sn.c, sn.dj));
      snap_out->Ej_new = St<T>::to_d(axpy_st<T>(Ej, cuj, sn.Ej));
      snap_out->dj_new =
          cmul(sn.dj, rdiv(1.0, make_double2(1.0 - sn.alpha * sn.dj.x, -sn.alpha * sn.dj.y)));
      snap_out->gm0_new = St<T>::to_d(axpy_st<T>(gm0j, cu_m0, St<T>::to_d(St<T>::from_d(sn.dj))));
      // the history (the term count stays in the snapshots)
      const int n = *n_flips;
      if (n < flip_cap) {
        flips[2 * n] = sn.j;
        flips[2 * n + 1] = sn.e_new;
      } else {
        atomicOr(status, GFO_STATUS_HISTORY_FULL);
      }
      *n_flips = n + 1;
    } else if (sn.pad1) {
      atomicOr(status, GFO_STATUS_SINGULAR);
    }
    gfo_pick rec = pk;
    if (rec.pixel >= 0) {
      rec.fom_new = scores_prev[rec.pixel * g.n_eps + rec.eps_idx];
      rec.dfom = rec.fom_new - fom;
    }
    *pick_out = rec;
  }
}

template <typename T, int PPL, int B>
__global__ __launch_bounds__(256) void k_move(
    Geo g, int has_prev, int flushed, const Snap* __restrict__ snap_prev,
    Snap* __restrict__ snap_out, const double* __restrict__ scores_prev,
    const double* __restrict__ partial_prev, const int* __restrict__ pfirst_prev, int nblk_prev,
    int bpix_prev, double* __restrict__ scores_next, double* __restrict__ partial_next,
    int* __restrict__ pfirst_next, const T* __restrict__ emon_prev, T* __restrict__ emon_next,
    uint32_t mask, double tau, gfo_pick* __restrict__ pick_out, T* __restrict__ G,
    T* __restrict__ E, double2* __restrict__ diag64, uint8_t* __restrict__ eps_idx,
    const int32_t* __restrict__ count, int32_t* __restrict__ flips, int flip_cap,
    int32_t* __restrict__ n_flips, int32_t* __restrict__ status, T* __restrict__ CUs,
    T* __restrict__ Vs) {
  move_body<T, PPL, B>(g, has_prev, flushed, snap_prev, snap_out, scores_prev, partial_prev,
                       pfirst_prev, nblk_prev, bpix_prev, scores_next, partial_next, pfirst_next,
                       emon_prev, emon_next, mask, tau, pick_out, G, E, diag64, eps_idx, count,
                       flips, flip_cap, n_flips, status, CUs, Vs);
}

// After move t of a one-kernel loop (its last, or before a flush): the move's
// pivot values, the fields at the monitors and the term count reach memory.
template <typename T>
__device__ __forceinline__ void move_finish_body(const Geo& g, const Snap* __restrict__ snap_last,
                                                 const T* __restrict__ emon_last, T* __restrict__ G,
                                                 T* __restrict__ E, double2* __restrict__ diag64,
                                                 uint8_t* __restrict__ eps_idx,
                                                 int32_t* __restrict__ count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < g.nmon) E[g.N + t] = emon_last[t];
  if (t == 0) {
    const Snap sn = *snap_last;
    *count = sn.cnt_after;
    if (sn.j >= 0) {
      E[sn.j] = St<T>::from_d(sn.Ej_new);
      diag64[sn.j] = sn.dj_new;
      eps_idx[sn.j] = (uint8_t)sn.e_new;
      G[g_off(g, g.N + g.m0, sn.j)] = St<T>::from_d(sn.gm0_new);
    }
  }
}

template <typename T>
__global__ void k_move_finish(Geo g, const Snap* __restrict__ snap_last,
                              const T* __restrict__ emon_last, T* __restrict__ G,
                              T* __restrict__ E, double2* __restrict__ diag64,
                              uint8_t* __restrict__ eps_idx, int32_t* __restrict__ count) {
  move_finish_body<T>(g, snap_last, emon_last, G, E, diag64, eps_idx, count);
}

template <typename T>
hipError_t launch_apply_deferred(const Geo& g, gfo_state* st, const Layout& L, const gfo_pick* pick,
                                 hipStream_t s) {
  char* w = (char*)st->work;
  Snap* snap = (Snap*)(w + L.snap);
  int32_t* count = (int32_t*)(w + L.dl_hdr);
  T* cu = (T*)(w + L.cu);
  T* v = (T*)(w + L.v);
  T* emon = (T*)(w + L.emon);
  const int64_t n = (int64_t)gather_mpad(g) + g.ld;
  hipLaunchKernelGGL((gather_batch(st->delay) == 16 ? k_gather_dl<T, 16> : k_gather_dl<T, 32>),
                     dim3((unsigned)((n + kGatherElems - 1) / kGatherElems)), dim3(256), 0, s, g, pick,
                     (const T*)st->G, (const T*)st->E, (const double2*)st->diag64,
                     (const uint8_t*)st->eps_idx, (const int32_t*)count, snap, (T*)(w + L.dl_CUs),
                     (T*)(w + L.dl_Vs), cu, v, emon);
  return launch_fused_finish<T>(g, st, L, s);
}

template <typename T>
hipError_t launch_fused_finish(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s) {
  char* w = (char*)st->work;
  const int64_t nx = g.R > g.ld ? (int64_t)g.R : g.ld;
  hipLaunchKernelGGL(k_mon_dl<T>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, g, (const Snap*)(w + L.snap),
                     (const T*)(w + L.cu), (const T*)(w + L.v), (const T*)(w + L.emon), (T*)st->G,
                     (T*)st->E, (double2*)st->diag64, st->eps_idx, st->flips, st->flip_cap,
                     st->n_flips, st->status, (int32_t*)(w + L.dl_hdr));
  return note_hip(hipGetLastError());
}

template <typename T>
hipError_t launch_fused_move(const Geo& g, gfo_state* st, const Layout& L, int apply_prev,
                             uint32_t mask, double tau, gfo_pick* pick_out, bool flush_between,
                             hipStream_t s) {
  char* w = (char*)st->work;
  Snap* snap = (Snap*)(w + L.snap);
  int32_t* count = (int32_t*)(w + L.dl_hdr);
  T* cu = (T*)(w + L.cu);
  T* v = (T*)(w + L.v);
  T* emon = (T*)(w + L.emon);
  double* scores = (double*)(w + L.scores);
  double* partial = (double*)(w + L.partial);
  int* pfirst = (int*)(w + L.pfirst);
  const int nblk = (g.N + kScoreThreads - 1) / kScoreThreads;
  const int64_t nx = g.R > g.ld ? (int64_t)g.R : g.ld;
  hipLaunchKernelGGL(k_mon_score<T>, dim3((unsigned)((nx + kScoreThreads - 1) / kScoreThreads)),
                     dim3(kScoreThreads), 0, s, g, apply_prev, (const Snap*)snap, (const T*)cu,
                     (const T*)v, (const T*)emon, (T*)st->G, (T*)st->E, (double2*)st->diag64,
                     st->eps_idx, st->flips, st->flip_cap, st->n_flips, st->status, count, mask,
                     tau, scores, partial, pfirst, nblk);
  if (flush_between) {
    const hipError_t e = launch_flush(g, st, L, s);
    if (e != hipSuccess) return e;
  }
  const int64_t n = (int64_t)gather_mpad(g) + g.ld;
  hipLaunchKernelGGL((gather_batch(st->delay) == 16 ? k_select_gather<T, 16> : k_select_gather<T, 32>),
                     dim3((unsigned)((n + kGatherElems - 1) / kGatherElems)),
                     dim3(256), 0, s, g,
                     (const double*)scores, (const double*)partial, (const int*)pfirst, nblk, tau,
                     pick_out,
                     (const T*)st->G, (const T*)st->E, (const double2*)st->diag64,
                     (const uint8_t*)st->eps_idx, (const int32_t*)count, snap, (T*)(w + L.dl_CUs),
                     (T*)(w + L.dl_Vs), cu, v, emon);
  return note_hip(hipGetLastError());
}

// The one-kernel loop serves shapes whose pixels fit kScoreMaxBlocks summaries
// of kGatherElems pixels.
bool one_kernel_loop(const Geo& g) {
  return (g.N + kGatherElems - 1) / kGatherElems <= kScoreMaxBlocks;
}

// One-kernel loop (k_move): move t of a call reads the buffer set t % 2 and
// writes the other; `flushed`: a flush ran since the previous move.
template <typename T>
hipError_t launch_move(const Geo& g, gfo_state* st, const Layout& L, int t, int flushed,
                       uint32_t mask, double tau, gfo_pick* pick_out, hipStream_t s) {
  char* w = (char*)st->work;
  Snap* snaps[2] = {(Snap*)(w + L.snap), (Snap*)(w + L.snap2)};
  T* emons[2] = {(T*)(w + L.emon), (T*)(w + L.emon2)};
  double* scores[2] = {(double*)(w + L.scores), (double*)(w + L.scores2)};
  double* partial[2] = {(double*)(w + L.partial), (double*)(w + L.partial2)};
  int* pfirst[2] = {(int*)(w + L.pfirst), (int*)(w + L.pfirst2)};
  const int a = t & 1, b = a ^ 1;
  // move 0 picks from the scoring kernel's summaries (kScoreThreads pixels each)
  const int bpix = t == 0 ? kScoreThreads : kGatherElems;
  const int nblk = (g.N + bpix - 1) / bpix;
  const int64_t n = (int64_t)gather_mpad(g) + g.ld;
  // summaries per lane: 4 while the grid has at most 256 of 64 pixels
  const bool small = (g.N + kGatherElems - 1) / kGatherElems <= 4 * 64;
  const bool b16 = gather_batch(st->delay) == 16;
  hipLaunchKernelGGL((small ? (b16 ? k_move<T, 4, 16> : k_move<T, 4, 32>)
                            : (b16 ? k_move<T, kPickPerLane, 16> : k_move<T, kPickPerLane, 32>)),
                     dim3((unsigned)((n + kGatherElems - 1) / kGatherElems)), dim3(256), 0,
                     s, g, t > 0 ? 1 : 0, flushed, (const Snap*)snaps[b], snaps[a],
                     (const double*)scores[a], (const double*)partial[a], (const int*)pfirst[a], nblk,
                     bpix, scores[b], partial[b], pfirst[b], (const T*)emons[b], emons[a], mask, tau,
                     pick_out, (T*)st->G, (T*)st->E, (double2*)st->diag64, st->eps_idx,
                     (const int32_t*)(w + L.dl_hdr), st->flips, st->flip_cap, st->n_flips,
                     st->status, (T*)(w + L.dl_CUs), (T*)(w + L.dl_Vs));
  return note_hip(hipGetLastError());
}

// After move t of a one-kernel loop: its last, or one before a flush.
template <typename T>
hipError_t launch_move_finish(const Geo& g, gfo_state* st, const Layout& L, int t, hipStream_t s) {
  char* w = (char*)st->work;
  const int a = t & 1;
  const Snap* snap = (const Snap*)(w + (a ? L.snap2 : L.snap));
  const T* emon = (const T*)(w + (a ? L.emon2 : L.emon));
  hipLaunchKernelGGL(k_move_finish<T>, dim3((unsigned)((g.nmon + 255) / 256)), dim3(256), 0, s, g,
                     snap, emon, (T*)st->G, (T*)st->E, (double2*)st->diag64, st->eps_idx,
                     (int32_t*)(w + L.dl_hdr));
  return note_hip(hipGetLastError());
}

// Scores of the current state into the first buffer set (the start of a
// one-kernel loop).
template <typename T>
hipError_t launch_move_scores(const Geo& g, gfo_state* st, const Layout& L, uint32_t mask,
                              double tau, hipStream_t s) {
  char* w = (char*)st->work;
  const int nblk = (g.N + kScoreThreads - 1) / kScoreThreads;
  const int64_t nx = g.R > g.ld ? (int64_t)g.R : g.ld;
  hipLaunchKernelGGL(k_mon_score<T>, dim3((unsigned)((nx + kScoreThreads - 1) / kScoreThreads)),
                     dim3(kScoreThreads), 0, s, g, 0, (const Snap*)(w + L.snap),
                     (const T*)(w + L.cu), (const T*)(w + L.v), (const T*)(w + L.emon), (T*)st->G,
                     (T*)st->E, (double2*)st->diag64, st->eps_idx, st->flips, st->flip_cap,
                     st->n_flips, st->status, (int32_t*)(w + L.dl_hdr), mask, tau,
                     (double*)(w + L.scores), (double*)(w + L.partial), (int*)(w + L.pfirst), nblk);
  return note_hip(hipGetLastError());
}

// ------------------------------------------------------------------ grouped launches
// The one-kernel loop of many jobs at once: workgroup (x, y) runs workgroup x
// of job y's own kernel with job y's arguments from the table (the same bodies,
// so every job's moves and state are bit for bit those of its own calls);
// workgroups past a job's count return at once.
int gather_move_workgroups(const Geo& g) {
  const int64_t n = (int64_t)gather_mpad(g) + g.ld;
  return (int)((n + kGatherElems - 1) / kGatherElems);
}

bool move_small_grid(const Geo& g) { return (g.N + kGatherElems - 1) / kGatherElems <= 4 * 64; }

JobEntry make_job_entry(const Geo& g, const gfo_state* st, const Layout& L, uint32_t mask,
                        double tau) {
  JobEntry je = {};
  je.g = g;
  je.G = st->G;
  je.E = st->E;
  je.diag64 = (double2*)st->diag64;
  je.eps_idx = st->eps_idx;
  je.flips = st->flips;
  je.n_flips = st->n_flips;
  je.status = st->status;
  je.work = (char*)st->work;
  je.snap = L.snap;
  je.snap2 = L.snap2;
  je.emon = L.emon;
  je.emon2 = L.emon2;
  je.scores = L.scores;
  je.scores2 = L.scores2;
  je.partial = L.partial;
  je.partial2 = L.partial2;
  je.pfirst = L.pfirst;
  je.pfirst2 = L.pfirst2;
  je.cu = L.cu;
  je.v = L.v;
  je.dl_hdr = L.dl_hdr;
  je.dl_CUs = L.dl_CUs;
  je.dl_Vs = L.dl_Vs;
  je.picks = L.picks;
  je.tau = tau;
  je.mask = mask;
  je.flip_cap = st->flip_cap;
  const int64_t nx = g.R > g.ld ? (int64_t)g.R : g.ld;
  je.n_score_wg = (int)((nx + kScoreThreads - 1) / kScoreThreads);
  je.n_move_wg = gather_move_workgroups(g);
  je.n_finish_wg = (g.nmon + 255) / 256;
  je.nblk0 = (g.N + kScoreThreads - 1) / kScoreThreads;
  je.nblkg = (g.N + kGatherElems - 1) / kGatherElems;
  return je;
}

template <typename T>
__global__ __launch_bounds__(kScoreThreads) void k_mon_score_table(const JobEntry* __restrict__ tab) {
  const JobEntry* je = tab + blockIdx.y;
  if ((int)blockIdx.x >= je->n_score_wg) return;
  const Geo g = je->g;
  char* w = je->work;
  mon_score_body<T>(g, 0, (const Snap*)(w + je->snap), (const T*)(w + je->cu),
                    (const T*)(w + je->v), (const T*)(w + je->emon), (T*)je->G, (T*)je->E,
                    je->diag64, je->eps_idx, je->flips, je->flip_cap, je->n_flips, je->status,
                    (int32_t*)(w + je->dl_hdr), je->mask, je->tau, (double*)(w + je->scores),
                    (double*)(w + je->partial), (int*)(w + je->pfirst), je->nblk0);
}

template <typename T, int PPL, int B>
__global__ __launch_bounds__(256) void k_move_table(const JobEntry* __restrict__ tab, int t,
                                                    uint64_t flushed_mask) {
  const JobEntry* je = tab + blockIdx.y;
  if ((int)blockIdx.x >= je->n_move_wg) return;
  const Geo g = je->g;
  char* w = je->work;
  const int a = t & 1;
  const int64_t snap_a = a ? je->snap2 : je->snap, snap_b = a ? je->snap : je->snap2;
  const int64_t emon_a = a ? je->emon2 : je->emon, emon_b = a ? je->emon : je->emon2;
  const int64_t sc_a = a ? je->scores2 : je->scores, sc_b = a ? je->scores : je->scores2;
  const int64_t pa_a = a ? je->partial2 : je->partial, pa_b = a ? je->partial : je->partial2;
  const int64_t pf_a = a ? je->pfirst2 : je->pfirst, pf_b = a ? je->pfirst : je->pfirst2;
  move_body<T, PPL, B>(g, t > 0 ? 1 : 0, (int)((flushed_mask >> blockIdx.y) & 1u),
                       (const Snap*)(w + snap_b), (Snap*)(w + snap_a), (const double*)(w + sc_a),
                       (const double*)(w + pa_a), (const int*)(w + pf_a),
                       t == 0 ? je->nblk0 : je->nblkg, t == 0 ? kScoreThreads : kGatherElems,
                       (double*)(w + sc_b), (double*)(w + pa_b), (int*)(w + pf_b),
                       (const T*)(w + emon_b), (T*)(w + emon_a), je->mask, je->tau,
                       (gfo_pick*)(w + je->picks), (T*)je->G, (T*)je->E, je->diag64, je->eps_idx,
                       (const int32_t*)(w + je->dl_hdr), je->flips, je->flip_cap, je->n_flips,
                       je->status, (T*)(w + je->dl_CUs), (T*)(w + je->dl_Vs));
}

template <typename T>
__global__ void k_move_finish_table(const JobEntry* __restrict__ tab, int t) {
  const JobEntry* je = tab + blockIdx.y;
  if ((int)blockIdx.x >= je->n_finish_wg) return;
  const Geo g = je->g;
  char* w = je->work;
  const int a = t & 1;
  move_finish_body<T>(g, (const Snap*)(w + (a ? je->snap2 : je->snap)),
                      (const T*)(w + (a ? je->emon2 : je->emon)), (T*)je->G, (T*)je->E,
                      je->diag64, je->eps_idx, (int32_t*)(w + je->dl_hdr));
}

template <typename T>
hipError_t launch_table_scores(const JobEntry* tab, int n_jobs, int max_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_mon_score_table<T>, dim3((unsigned)max_wg, (unsigned)n_jobs),
                     dim3(kScoreThreads), 0, s, tab);
  return note_hip(hipGetLastError());
}

template <typename T>
hipError_t launch_table_move(const JobEntry* tab, int n_jobs, int max_wg, int t, uint64_t flushed,
                             bool small, int batch, hipStream_t s) {
  const dim3 grid((unsigned)max_wg, (unsigned)n_jobs);
  const bool b16 = batch == 16;
  hipLaunchKernelGGL((small ? (b16 ? k_move_table<T, 4, 16> : k_move_table<T, 4, 32>)
                            : (b16 ? k_move_table<T, kPickPerLane, 16>
                                   : k_move_table<T, kPickPerLane, 32>)),
                     grid, dim3(256), 0, s, tab, t, flushed);
  return note_hip(hipGetLastError());
}

template <typename T>
hipError_t launch_table_finish(const JobEntry* tab, int n_jobs, int max_wg, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_move_finish_table<T>, dim3((unsigned)max_wg, (unsigned)n_jobs), dim3(256), 0,
                     s, tab, t);
  return note_hip(hipGetLastError());
}

template hipError_t launch_table_scores<float2>(const JobEntry*, int, int, hipStream_t);
template hipError_t launch_table_scores<double2>(const JobEntry*, int, int, hipStream_t);
template hipError_t launch_table_move<float2>(const JobEntry*, int, int, int, uint64_t, bool, int,
                                              hipStream_t);
template hipError_t launch_table_move<double2>(const JobEntry*, int, int, int, uint64_t, bool, int,
                                               hipStream_t);
template hipError_t launch_table_finish<float2>(const JobEntry*, int, int, int, hipStream_t);
template hipError_t launch_table_finish<double2>(const JobEntry*, int, int, int, hipStream_t);

template hipError_t launch_move<float2>(const Geo&, gfo_state*, const Layout&, int, int, uint32_t,
                                        double, gfo_pick*, hipStream_t);
template hipError_t launch_move<double2>(const Geo&, gfo_state*, const Layout&, int, int, uint32_t,
                                         double, gfo_pick*, hipStream_t);
template hipError_t launch_move_finish<float2>(const Geo&, gfo_state*, const Layout&, int, hipStream_t);
template hipError_t launch_move_finish<double2>(const Geo&, gfo_state*, const Layout&, int, hipStream_t);
template hipError_t launch_move_scores<float2>(const Geo&, gfo_state*, const Layout&, uint32_t, double,
                                               hipStream_t);
template hipError_t launch_move_scores<double2>(const Geo&, gfo_state*, const Layout&, uint32_t,
                                                double, hipStream_t);

template hipError_t launch_fused_move<float2>(const Geo&, gfo_state*, const Layout&, int, uint32_t,
                                              double, gfo_pick*, bool, hipStream_t);
template hipError_t launch_fused_move<double2>(const Geo&, gfo_state*, const Layout&, int, uint32_t,
                                               double, gfo_pick*, bool, hipStream_t);
template hipError_t launch_fused_finish<float2>(const Geo&, gfo_state*, const Layout&, hipStream_t);
template hipError_t launch_fused_finish<double2>(const Geo&, gfo_state*, const Layout&, hipStream_t);

template hipError_t launch_apply_deferred<float2>(const Geo&, gfo_state*, const Layout&,
                                                  const gfo_pick*, hipStream_t);
template hipError_t launch_apply_deferred<double2>(const Geo&, gfo_state*, const Layout&,
                                                   const gfo_pick*, hipStream_t);

}  // namespace gfo
