// Deferred rank-1 updates.  Eq. form10 applied move by move gives
//   G_t = G_base + sum_{s < t} cu_s v_s^T,   cu_s = c_s G_s[:, j_s],  v_s = G_s[j_s, :],
// so the design block can be brought up to date later, in one rank-r product,
// while everything the scores read (E, diag64, the monitor rows) is updated at
// once.  Column j and row j of the current matrix are the base entries plus the
// pending terms.
#include "gfo_internal.hpp"

namespace gfo {

// Thread i: u_i = G_t[i, j] (base + pending, rows < N; monitor rows are current),
// v_i = G_t[j, i]; stores term `slot`; E_i += c u_i E_j; diag64_i += c u_i v_i.
template <typename T>
__global__ void k_gather_dl(Geo g, const Snap* __restrict__ snap, const T* __restrict__ G,
                            T* __restrict__ E, double2* __restrict__ diag64, T* __restrict__ CU,
                            T* __restrict__ V) {
  const int j = snap->j;
  if (j < 0) return;
  const int slot = snap->slot;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double2 c = snap->c;
  double2 cu_d = make_double2(0.0, 0.0);
  if (i < g.R) {
    double2 u;
    if (i == j) {
      u = snap->dj;
    } else {
      u = St<T>::to_d(G[i * g.ld + j]);
      if (i < g.N)
        for (int s = 0; s < slot; ++s)
          u = cadd(u, cmul(St<T>::to_d(CU[(int64_t)s * g.R + i]),
                           St<T>::to_d(V[(int64_t)s * g.ld + j])));
    }
    cu_d = cmul(c, u);
    CU[(int64_t)slot * g.R + i] = St<T>::from_d(cu_d);
    E[i] = St<T>::from_d(cadd(St<T>::to_d(E[i]), cmul(cu_d, snap->Ej)));
  }
  if (i < g.ld) {
    if (i < g.N) {
      double2 v;
      if (i == j) {
        v = snap->dj;
      } else {
        v = St<T>::to_d(G[(int64_t)j * g.ld + i]);
        for (int s = 0; s < slot; ++s)
          v = cadd(v, cmul(St<T>::to_d(CU[(int64_t)s * g.R + j]),
                           St<T>::to_d(V[(int64_t)s * g.ld + i])));
      }
      V[(int64_t)slot * g.ld + i] = St<T>::from_d(v);
      if (i == j) {
        const double2 d = snap->dj;
        diag64[j] = cmul(d, rdiv(1.0, make_double2(1.0 - snap->alpha * d.x, -snap->alpha * d.y)));
      } else {
        diag64[i] = cadd(diag64[i], cmul(cu_d, v));
      }
    } else {
      V[(int64_t)slot * g.ld + i] = St<T>::from_d(make_double2(0.0, 0.0));
    }
  }
}

// Monitor rows stay current: G[N+m, q] += cu[N+m] v[q].
template <typename T>
__global__ void k_mon_dl(Geo g, const Snap* __restrict__ snap, const T* __restrict__ CU,
                         const T* __restrict__ V, T* __restrict__ G) {
  if (snap->j < 0) return;
  const int slot = snap->slot;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.ld) return;
  const double2 vq = St<T>::to_d(V[(int64_t)slot * g.ld + q]);
  for (int m = blockIdx.y; m < g.nmon; m += gridDim.y) {
    const int64_t r = g.N + m;
    const double2 cu = St<T>::to_d(CU[(int64_t)slot * g.R + r]);
    T* p = G + r * g.ld + q;
    *p = St<T>::from_d(cadd(St<T>::to_d(*p), cmul(cu, vq)));
  }
}

// FP32 operands of the flush, same lane order as the rank-k product:
// A[r][kappa] (r < N): kappa < 64 Re cu_kappa[r], kappa >= 64 Im cu;
// B[q][out][kappa]: out 0 = [Re v ; -Im v], out 1 = [Im v ; Re v]; slots >= count are zero.
__global__ void k_dl_packA(Geo g, const int32_t* __restrict__ count, const float2* __restrict__ CU,
                           float* __restrict__ A) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.N) return;
  const int n = *count;
  constexpr int KP = GFO_MAX_DELAY;
  for (int s = 0; s < KP; ++s) {
    const float2 v = s < n ? CU[(int64_t)s * g.R + r] : make_float2(0.f, 0.f);
    A[(int64_t)r * 2 * KP + s] = v.x;
    A[(int64_t)r * 2 * KP + KP + s] = v.y;
  }
}

__global__ void k_dl_packB(Geo g, const int32_t* __restrict__ count, const float2* __restrict__ V,
                           float* __restrict__ B) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.ld) return;
  const int n = *count;
  constexpr int KP = GFO_MAX_DELAY;
  const int64_t base = q * 4 * KP;
  for (int s = 0; s < KP; ++s) {
    const float2 w = s < n ? V[(int64_t)s * g.ld + q] : make_float2(0.f, 0.f);
    B[base + s] = w.x;
    B[base + KP + s] = -w.y;
    B[base + 2 * KP + s] = w.y;
    B[base + 3 * KP + s] = w.x;
  }
}

__global__ void k_dl_reset(int32_t* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count = 0;
}

hipError_t launch_dl_reset(const Geo&, gfo_state* st, const Layout& L, hipStream_t s) {
  hipLaunchKernelGGL(k_dl_reset, dim3(1), dim3(64), 0, s, (int32_t*)((char*)st->work + L.dl_hdr));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_deferred(const Geo& g, gfo_state* st, const Layout& L, const Snap* snap,
                                 hipStream_t s) {
  char* w = (char*)st->work;
  T* CU = (T*)(w + L.dl_CU);
  T* V = (T*)(w + L.dl_V);
  const int64_t n = g.R > g.ld ? (int64_t)g.R : g.ld;
  hipLaunchKernelGGL(k_gather_dl<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, snap,
                     (const T*)st->G, (T*)st->E, (double2*)st->diag64, CU, V);
  dim3 gm((unsigned)((g.ld + 255) / 256), (unsigned)(g.nmon < 65535 ? g.nmon : 65535));
  hipLaunchKernelGGL(k_mon_dl<T>, gm, dim3(256), 0, s, g, snap, (const T*)CU, (const T*)V,
                     (T*)st->G);
  return hipGetLastError();
}
template hipError_t launch_apply_deferred<float2>(const Geo&, gfo_state*, const Layout&,
                                                  const Snap*, hipStream_t);
template hipError_t launch_apply_deferred<double2>(const Geo&, gfo_state*, const Layout&,
                                                   const Snap*, hipStream_t);

hipError_t launch_flush(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s) {
  char* w = (char*)st->work;
  const int32_t* count = (const int32_t*)(w + L.dl_hdr);
  hipEvent_t before, after;
  k1_take_timing(&before, &after);
  hipError_t e;
  if (g.dtype == GFO_C64) {
    float* A = (float*)(w + L.dl_A);
    float* B = (float*)(w + L.dl_B);
    hipLaunchKernelGGL(k_dl_packA, dim3((g.N + 255) / 256), dim3(256), 0, s, g, count,
                       (const float2*)(w + L.dl_CU), A);
    hipLaunchKernelGGL(k_dl_packB, dim3((unsigned)((g.ld + 255) / 256)), dim3(256), 0, s, g, count,
                       (const float2*)(w + L.dl_V), B);
    if (before && hipEventRecord(before, s) != hipSuccess) return hipErrorUnknown;
    e = launch_mfma_update_f32_64(g.N, g.ld, count, A, B, (float2*)st->G, s);
  } else {
    if (before && hipEventRecord(before, s) != hipSuccess) return hipErrorUnknown;
    e = launch_zgemm_update_f64(g, count, (const double2*)(w + L.dl_CU),
                                (const double2*)(w + L.dl_V), (double2*)st->G, s);
  }
  if (e != hipSuccess) return e;
  if (after && hipEventRecord(after, s) != hipSuccess) return hipErrorUnknown;
  hipLaunchKernelGGL(k_dl_reset, dim3(1), dim3(64), 0, s, (int32_t*)(w + L.dl_hdr));
  return hipGetLastError();
}

}  // namespace gfo
