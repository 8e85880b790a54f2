// init_G0 kernels: FP64 Hankel table over pixel offsets, fill of the design
// block by translation invariance, direct evaluation of the monitor rows, the
// incident plane wave and the FP64 diagonal.
//
// Free-space 2-D kernel (vacuum reference structure, paper Sec. II/IV):
//   h^2 (i/4) H0^(1)(k0 r) = h^2/4 * (-Y0(k0 r) + i J0(k0 r))
// Self term over the equal-area disk a = h/sqrt(pi):
//   (i pi a / (2 k0)) H1^(1)(k0 a) - 1/k0^2
//     = (-pi a Y1(k0 a)/(2 k0) - 1/k0^2) + i (pi a J1(k0 a)/(2 k0)).
// J0/Y0/J1/Y1 are the FP64 device Bessel functions of the ROCm math library.
#include "gfo_internal.hpp"

namespace gfo {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 kernel_h2g(double r, const Geo& g) {
  double x = g.k0 * r;
  double s = 0.25 * g.h * g.h;
  return make_double2(-s * y0(x), s * j0(x));
}

__device__ __forceinline__ double2 self_term(const Geo& g) {
  const double pi = 3.14159265358979323846;
  double a = g.h / sqrt(pi);
  double x = g.k0 * a;
  double f = pi * a / (2.0 * g.k0);
  return make_double2(-f * y1(x) - 1.0 / g.k0sq, f * j1(x));
}

// table[dy * nx + dx] = G0 between pixels offset by (dy, dx) rows/cols
__global__ void k_init_table(Geo g, double2* __restrict__ table) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.ny * g.nx) return;
  int dy = i / g.nx, dx = i - (i / g.nx) * g.nx;
  double2 v;
  if (i == 0) {
    v = self_term(g);
  } else {
    double r = g.h * sqrt((double)dx * dx + (double)dy * dy);
    v = kernel_h2g(r, g);
  }
  table[i] = v;
}

// Design block: G[p, q] = table[|iy_p - iy_q|, |ix_p - ix_q|]; columns >= N zeroed.
// A thread writes VN = 16 / sizeof(T) consecutive columns of a row with one
// 16-byte non-temporal store; the workgroups of grid row y take the rows
// y, y + gridDim.y, ...  With `upper`, stores that lie wholly below the
// diagonal are skipped (deferred mode reads the design block from its upper
// triangle; the caller marks the lower one out of date).
template <typename T>
__global__ void k_fill_design(Geo g, T* __restrict__ G, const double2* __restrict__ table,
                              int upper) {
  constexpr int VN = 16 / (int)sizeof(T);
  const int64_t q0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VN;
  if (q0 >= g.ld) return;
  int iyq[VN], ixq[VN];
#pragma unroll
  for (int v = 0; v < VN; ++v) {
    iyq[v] = (int)((q0 + v) / g.nx);
    ixq[v] = (int)(q0 + v - (int64_t)iyq[v] * g.nx);
  }
  // with `upper`, rows past the workgroup's last column hold nothing to write
  const int64_t wg_end = ((int64_t)blockIdx.x + 1) * blockDim.x * VN;
  const int p_end = upper && wg_end < g.N ? (int)wg_end : g.N;
  // two rows per step: both rows' table reads are in flight before the stores
  // (one row at a time: init_G0 329 us at 128 x 128; two: 291 us; four or eight:
  // no faster)
  constexpr int RB = 2;
  for (int p0 = blockIdx.y; p0 < p_end; p0 += RB * gridDim.y) {
    double2 d[RB][VN];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int p = p0 + r * gridDim.y;
      const int iyp = p / g.nx, ixp = p - (p / g.nx) * g.nx;
#pragma unroll
      for (int v = 0; v < VN; ++v) {
        d[r][v] = make_double2(0.0, 0.0);
        if (p < p_end && q0 + v < g.N) d[r][v] = table[abs(iyp - iyq[v]) * g.nx + abs(ixp - ixq[v])];
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int p = p0 + r * gridDim.y;
      if (p >= p_end || (upper && q0 + VN - 1 < p)) continue;
      T* dst = G + g_off(g, p, q0);   // packed: q0 >= 64 (p / 64) here (upper)
      if constexpr (VN == 2) {
        const float2 a = St<T>::from_d(d[r][0]), b = St<T>::from_d(d[r][1]);
        __builtin_nontemporal_store(f32x4{a.x, a.y, b.x, b.y}, (f32x4*)dst);
      } else {
        __builtin_nontemporal_store(f64x2{d[r][0].x, d[r][0].y}, (f64x2*)dst);
      }
    }
  }
}

// Monitor rows: direct FP64 evaluation.
template <typename T>
__global__ void k_fill_monitors(Geo g, T* __restrict__ G, const double* __restrict__ mon_xy) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.ld) return;
  for (int m = blockIdx.y; m < g.nmon; m += gridDim.y) {
    T out;
    if (q < g.N) {
      int iyq = (int)(q / g.nx), ixq = (int)(q - (int64_t)iyq * g.nx);
      double xq = (ixq - 0.5 * (g.nx - 1)) * g.h;
      double yq = (iyq - 0.5 * (g.ny - 1)) * g.h;
      double dx = mon_xy[2 * m] - xq, dy = mon_xy[2 * m + 1] - yq;
      out = St<T>::from_d(kernel_h2g(sqrt(dx * dx + dy * dy), g));
    } else {
      out = St<T>::from_d(make_double2(0.0, 0.0));
    }
    G[g_off(g, g.N + m, q)] = out;
  }
}

// E = exp(i k0 y) on every row; diag64, eps_idx, counters.
template <typename T>
__global__ void k_init_vectors(Geo g, T* __restrict__ E, double2* __restrict__ diag64,
                               uint8_t* __restrict__ eps_idx, const double* __restrict__ mon_xy,
                               const double2* __restrict__ table, int32_t* n_flips,
                               int32_t* status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.R) {
    double y;
    if (i < g.N) {
      int iy = i / g.nx;
      y = (iy - 0.5 * (g.ny - 1)) * g.h;
    } else {
      y = mon_xy[2 * (i - g.N) + 1];
    }
    double s, c;
    sincos(g.k0 * y, &s, &c);
    E[i] = St<T>::from_d(make_double2(c, s));
  }
  if (i < g.N) {
    diag64[i] = table[0];
    eps_idx[i] = (uint8_t)g.bg_idx;
  }
  if (i == 0) {
    *n_flips = 0;
    *status = 0;
  }
}

template <typename T>
static hipError_t init_typed(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s) {
  char* w = (char*)st->work;
  double2* table = (double2*)(w + L.table);
  double* mon = (double*)(w + L.mon_xy);
  T* G = (T*)st->G;
  int nt = g.ny * g.nx;
  hipLaunchKernelGGL(k_init_table, dim3((nt + 255) / 256), dim3(256), 0, s, g, table);
  dim3 blk(256);
  constexpr int VN = 16 / (int)sizeof(T);
  // a few rows per workgroup: workgroup dispatch, not the stores, bounds one row each
  dim3 grd((unsigned)((g.ld + 256 * VN - 1) / (256 * VN)), (unsigned)(g.N < 2048 ? g.N : 2048));
  hipLaunchKernelGGL(k_fill_design<T>, grd, blk, 0, s, g, G, (const double2*)table,
                     g.upper);
  if (g.nmon > 0) {
    dim3 grm((unsigned)((g.ld + 255) / 256), (unsigned)(g.nmon < 65535 ? g.nmon : 65535));
    hipLaunchKernelGGL(k_fill_monitors<T>, grm, blk, 0, s, g, G, (const double*)mon);
  }
  hipLaunchKernelGGL(k_init_vectors<T>, dim3((g.R + 255) / 256), dim3(256), 0, s, g, (T*)st->E,
                     (double2*)st->diag64, st->eps_idx, (const double*)mon, (const double2*)table,
                     st->n_flips, st->status);
  return note_hip(hipGetLastError());
}

hipError_t launch_init(const Geo& g, gfo_state* st, const Layout& L, hipStream_t s) {
  if (g.dtype == GFO_C64) return init_typed<float2>(g, st, L, s);
  return init_typed<double2>(g, st, L, s);
}

}  // namespace gfo
