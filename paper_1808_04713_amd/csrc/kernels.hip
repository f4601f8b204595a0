// Device kernels of the interface-problem solver for gfx950 (64-wide waves).
//
// Layouts: every vector family stores the right-hand-side index fastest
// (stride R).  Dual-slot arrays hold, per element, the type-1 edge modes that
// the jump operator C_1 touches; full-element arrays hold all n_e^2 vertex-
// basis coefficients of every element.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "kernels.hpp"

namespace hdp {

namespace {

constexpr int NT = 256;      // threads per block
constexpr int RC = 8;        // RHS columns per block in the slot kernels
constexpr int MMAX = 160;    // max dual slots per element (4 sides x 40 modes)
constexpr int NRMAX = 160;   // max coarse modes per element

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
  return make_float2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

template <class T2> struct Scal;
template <> struct Scal<double2> { using T = double; };
template <> struct Scal<float2> { using T = float; };

template <class T2> __device__ __forceinline__ T2 mk(double x, double y);
template <> __device__ __forceinline__ double2 mk<double2>(double x, double y) { return make_double2(x, y); }
template <> __device__ __forceinline__ float2 mk<float2>(double x, double y) { return make_float2(float(x), float(y)); }

// ---------------------------------------------------------------------------
// Slot kernels: one block per element (class-grouped order), RC RHS per block.
template <class T2, int MODE>
__global__ void __launch_bounds__(NT) k_slot_apply(
    const int* __restrict__ order, const int* __restrict__ elem_cls, const int* __restrict__ slot_off,
    const int* __restrict__ cm_off, const int* __restrict__ cls_m, const int* __restrict__ cls_nr,
    const int64_t* __restrict__ cls_op, const T2* __restrict__ op1, const typename Scal<T2>::T* __restrict__ se,
    const int64_t* __restrict__ cls_se, const int* __restrict__ slot_row, const double* __restrict__ slot_coef,
    const double* __restrict__ row_xinv, const T2* __restrict__ v, T2* __restrict__ X, T2* __restrict__ GL,
    int R) {
  using S = typename Scal<T2>::T;
  __shared__ T2 y[MMAX * RC];
  const int e = order[blockIdx.x];
  const int c = elem_cls[e];
  const int m = cls_m[c];
  const int nr = cls_nr[c];
  const int r0 = blockIdx.y * RC;
  const int rc = min(RC, R - r0);
  const int so = slot_off[e];
  for (int idx = threadIdx.x; idx < m * rc; idx += NT) {
    int s = idx / rc, r = idx - s * rc;
    int slot = so + s;
    int row = slot_row[slot];
    S f = S(slot_coef[slot]);
    if (MODE == 1) f *= S(row_xinv[row]);
    T2 a = v[(int64_t)row * R + r0 + r];
    y[s * RC + r] = mk<T2>(f * a.x, f * a.y);
  }
  __syncthreads();
  if (MODE == 0) {
    const int nrow = m + nr;
    const T2* A = op1 + cls_op[c];
    for (int idx = threadIdx.x; idx < nrow * rc; idx += NT) {
      int i = idx / rc, r = idx - i * rc;
      T2 acc = mk<T2>(0, 0);
      for (int kk = 0; kk < m; ++kk) acc = cfma(A[i + (int64_t)nrow * kk], y[kk * RC + r], acc);
      if (i < m) X[(int64_t)(so + i) * R + r0 + r] = acc;
      else GL[(int64_t)(cm_off[e] + i - m) * R + r0 + r] = acc;
    }
  } else {
    const S* A = se + cls_se[c];
    for (int idx = threadIdx.x; idx < m * rc; idx += NT) {
      int i = idx / rc, r = idx - i * rc;
      S ax = 0, ay = 0;
      for (int kk = 0; kk < m; ++kk) {
        S a = A[i + (int64_t)m * kk];
        T2 b = y[kk * RC + r];
        ax += a * b.x;
        ay += a * b.y;
      }
      X[(int64_t)(so + i) * R + r0 + r] = mk<T2>(ax, ay);
    }
  }
}

template <class T2>
__global__ void __launch_bounds__(NT) k_slot_coarse(
    const int* __restrict__ order, const int* __restrict__ elem_cls, const int* __restrict__ slot_off,
    const int* __restrict__ cm_off, const int* __restrict__ cls_m, const int* __restrict__ cls_nr,
    const int64_t* __restrict__ cls_phi, const T2* __restrict__ phi, const int* __restrict__ cm_dof,
    const T2* __restrict__ X, const double2* __restrict__ w, T2* __restrict__ Z, int R) {
  __shared__ T2 we[NRMAX * RC];
  const int e = order[blockIdx.x];
  const int c = elem_cls[e];
  const int m = cls_m[c], nr = cls_nr[c];
  const int r0 = blockIdx.y * RC;
  const int rc = min(RC, R - r0);
  const int co = cm_off[e], so = slot_off[e];
  for (int idx = threadIdx.x; idx < nr * rc; idx += NT) {
    int j = idx / rc, r = idx - j * rc;
    double2 a = w[(int64_t)cm_dof[co + j] * R + r0 + r];
    we[j * RC + r] = mk<T2>(a.x, a.y);
  }
  __syncthreads();
  const T2* P = phi + cls_phi[c];
  for (int idx = threadIdx.x; idx < m * rc; idx += NT) {
    int i = idx / rc, r = idx - i * rc;
    T2 acc = X[(int64_t)(so + i) * R + r0 + r];
    for (int j = 0; j < nr; ++j) acc = cfma(P[i + (int64_t)m * j], we[j * RC + r], acc);
    Z[(int64_t)(so + i) * R + r0 + r] = acc;
  }
}

template <class T2>
__global__ void k_rowgather(int nlam, const int* __restrict__ row_slot, const double* __restrict__ row_coef,
                            const double* __restrict__ row_xinv, const int64_t* __restrict__ slot_pos,
                            const T2* __restrict__ src, double2* __restrict__ u, int R) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nlam * R) return;
  int row = int(idx / R), r = int(idx - (int64_t)row * R);
  double ax = 0, ay = 0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    int slot = row_slot[2 * row + t];
    if (slot < 0) continue;
    int64_t pos = slot_pos ? slot_pos[slot] : slot;
    T2 a = src[pos * R + r];
    double cf = row_coef[2 * row + t];
    ax += cf * double(a.x);
    ay += cf * double(a.y);
  }
  if (row_xinv) {
    ax *= row_xinv[row];
    ay *= row_xinv[row];
  }
  u[idx] = make_double2(ax, ay);
}

template <class T2>
__global__ void k_assemble(int nK, const int* __restrict__ ptr, const int* __restrict__ list,
                           const T2* __restrict__ GL, const int64_t* __restrict__ cm_pos,
                           const double2* __restrict__ Bfull, double2* __restrict__ g, int R) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nK * R) return;
  int d = int(idx / R), r = int(idx - (int64_t)d * R);
  double ax = 0, ay = 0;
  for (int t = ptr[d]; t < ptr[d + 1]; ++t) {
    int i = list[t];
    if (GL) {
      T2 a = GL[(int64_t)i * R + r];
      ax += double(a.x);
      ay += double(a.y);
    }
    if (Bfull) {
      double2 b = Bfull[cm_pos[i] * R + r];
      ax += b.x;
      ay += b.y;
    }
  }
  g[idx] = make_double2(ax, ay);
}

// w = K^-1 g: one wavefront per row of the (symmetric) inverse, RHS in chunks of 8.
__global__ void __launch_bounds__(NT) k_coarse_gemv(int nK, const double2* __restrict__ Kinv,
                                                    const double2* __restrict__ g, double2* __restrict__ w,
                                                    int R) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (row >= nK) return;
  const double2* Kr = Kinv + (int64_t)row * nK;
  for (int r0 = 0; r0 < R; r0 += 8) {
    int rc = min(8, R - r0);
    double ax[8] = {0}, ay[8] = {0};
    for (int j = lane; j < nK; j += 64) {
      double2 a = Kr[j];
      for (int r = 0; r < rc; ++r) {
        double2 b = g[(int64_t)j * R + r0 + r];
        ax[r] += a.x * b.x - a.y * b.y;
        ay[r] += a.x * b.y + a.y * b.x;
      }
    }
    for (int r = 0; r < rc; ++r) {
      double sx = ax[r], sy = ay[r];
      for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_down(sx, off, 64);
        sy += __shfl_down(sy, off, 64);
      }
      if (lane == 0) w[(int64_t)row * R + r0 + r] = make_double2(sx, sy);
    }
  }
}

// ---------------------------------------------------------------------------
// Full-element separable solve X = Ex [(Ex^T Y Ey) ./ D] Ey^T, one block per (element, RHS).
__global__ void __launch_bounds__(NT) k_fdm(const int* __restrict__ elem_cls, const int64_t* __restrict__ dof_off,
                                            const int* __restrict__ cls_n, const int64_t* __restrict__ cls_E,
                                            const int64_t* __restrict__ cls_D, const double2* __restrict__ Ex,
                                            const double2* __restrict__ Ey, const double2* __restrict__ Dinv,
                                            const double2* __restrict__ in, double2* __restrict__ out, int R) {
  extern __shared__ double2 sm[];
  const int e = blockIdx.x;
  const int r = blockIdx.y;
  const int c = elem_cls[e];
  const int n = cls_n[c], n2 = n * n;
  double2* A = sm;
  double2* B = sm + n2;
  const double2* ex = Ex + cls_E[c];
  const double2* ey = Ey + cls_E[c];
  const double2* di = Dinv + cls_D[c];
  const int64_t base = dof_off[e];
  for (int t = threadIdx.x; t < n2; t += NT) A[t] = in[(base + t) * R + r];
  __syncthreads();
  // B = Ex^T A
  for (int t = threadIdx.x; t < n2; t += NT) {
    int i = t % n, j = t / n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(ex[k + n * i], A[k + n * j], acc);
    B[t] = acc;
  }
  __syncthreads();
  // A = (B Ey) .* Dinv
  for (int t = threadIdx.x; t < n2; t += NT) {
    int i = t % n, j = t / n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(B[i + n * k], ey[k + n * j], acc);
    A[t] = cmul(acc, di[t]);
  }
  __syncthreads();
  // B = Ex A
  for (int t = threadIdx.x; t < n2; t += NT) {
    int i = t % n, j = t / n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(ex[i + n * k], A[k + n * j], acc);
    B[t] = acc;
  }
  __syncthreads();
  // out = B Ey^T
  for (int t = threadIdx.x; t < n2; t += NT) {
    int i = t % n, j = t / n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(B[i + n * k], ey[j + n * k], acc);
    out[(base + t) * R + r] = acc;
  }
}

__global__ void k_zero_R(int E, const int* __restrict__ elem_cls, const int64_t* __restrict__ dof_off,
                         const int* __restrict__ cls_nr, const int* __restrict__ cls_R,
                         const int* __restrict__ r_modes, double2* __restrict__ X, int R) {
  int e = blockIdx.x;
  int c = elem_cls[e];
  int nr = cls_nr[c];
  const int* rm = r_modes + cls_R[c];
  for (int t = threadIdx.x; t < nr * R; t += blockDim.x) {
    int a = t / R, r = t - a * R;
    X[(dof_off[e] + rm[a]) * R + r] = make_double2(0, 0);
  }
}

// GL_e = Kc (X_e at the coarse modes): the element's share of -Phi^T y.
__global__ void k_extract_kc(const int* __restrict__ elem_cls, const int64_t* __restrict__ dof_off,
                             const int* __restrict__ cm_off, const int* __restrict__ cls_nr,
                             const int* __restrict__ cls_R, const int* __restrict__ r_modes,
                             const int64_t* __restrict__ cls_Kc, const double2* __restrict__ Kc,
                             const double2* __restrict__ X, double2* __restrict__ GL, int R) {
  __shared__ double2 cv[NRMAX];
  int e = blockIdx.x, r = blockIdx.y;
  int c = elem_cls[e];
  int nr = cls_nr[c];
  const int* rm = r_modes + cls_R[c];
  for (int a = threadIdx.x; a < nr; a += blockDim.x) cv[a] = X[(dof_off[e] + rm[a]) * R + r];
  __syncthreads();
  const double2* K = Kc + cls_Kc[c];
  for (int a = threadIdx.x; a < nr; a += blockDim.x) {
    double2 acc = make_double2(0, 0);
    for (int b = 0; b < nr; ++b) acc = cfma(K[a + nr * b], cv[b], acc);
    GL[(int64_t)(cm_off[e] + a) * R + r] = acc;
  }
}

// mu = Kc (c - T_e w); X -= G mu.  Afterwards X at the coarse modes equals T_e w.
__global__ void __launch_bounds__(NT) k_correct(const int* __restrict__ elem_cls, const int64_t* __restrict__ dof_off,
                                                const int* __restrict__ cm_off, const int* __restrict__ cls_n,
                                                const int* __restrict__ cls_nr, const int* __restrict__ cls_R,
                                                const int* __restrict__ r_modes, const int64_t* __restrict__ cls_Kc,
                                                const double2* __restrict__ Kc, const int64_t* __restrict__ cls_G,
                                                const double2* __restrict__ G, const int* __restrict__ cm_dof,
                                                double2* __restrict__ X, const double2* __restrict__ w, int R) {
  __shared__ double2 dv[NRMAX], mu[NRMAX];
  int e = blockIdx.x, r = blockIdx.y;
  int c = elem_cls[e];
  int n = cls_n[c], n2 = n * n, nr = cls_nr[c];
  const int* rm = r_modes + cls_R[c];
  const int64_t base = dof_off[e];
  for (int a = threadIdx.x; a < nr; a += blockDim.x) {
    double2 x = X[(base + rm[a]) * R + r];
    double2 ww = w[(int64_t)cm_dof[cm_off[e] + a] * R + r];
    dv[a] = make_double2(x.x - ww.x, x.y - ww.y);
  }
  __syncthreads();
  const double2* K = Kc + cls_Kc[c];
  for (int a = threadIdx.x; a < nr; a += blockDim.x) {
    double2 acc = make_double2(0, 0);
    for (int b = 0; b < nr; ++b) acc = cfma(K[a + nr * b], dv[b], acc);
    mu[a] = acc;
  }
  __syncthreads();
  const double2* Gc = G + cls_G[c];
  for (int t = threadIdx.x; t < n2; t += NT) {
    double2 acc = X[(base + t) * R + r];
    for (int a = 0; a < nr; ++a) {
      double2 gm = cmul(Gc[t + (int64_t)n2 * a], mu[a]);
      acc.x -= gm.x;
      acc.y -= gm.y;
    }
    X[(base + t) * R + r] = acc;
  }
}

// Y[pos(slot)] -= coef * nu[row(slot)]   (y_I = b_1 - C_1^T nu)
__global__ void k_sub_dual(int nslots, const int64_t* __restrict__ slot_pos, const int* __restrict__ slot_row,
                           const double* __restrict__ slot_coef, double2* __restrict__ Y,
                           const double2* __restrict__ nu, int R) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nslots * R) return;
  int s = int(idx / R), r = int(idx - (int64_t)s * R);
  double2 a = nu[(int64_t)slot_row[s] * R + r];
  double cf = slot_coef[s];
  double2& y = Y[slot_pos[s] * R + r];
  y.x -= cf * a.x;
  y.y -= cf * a.y;
}

// field = V X V^T at the GLL nodes of each element (V[i,a] = N~_a(t_i)).
__global__ void __launch_bounds__(NT) k_gll(const int* __restrict__ elem_cls, const int64_t* __restrict__ dof_off,
                                            const int* __restrict__ cls_n, const int64_t* __restrict__ cls_V,
                                            const double* __restrict__ V, const double2* __restrict__ X,
                                            double2* __restrict__ field, int R, int64_t rhs_stride) {
  extern __shared__ double2 sm[];
  int e = blockIdx.x, r = blockIdx.y;
  int c = elem_cls[e];
  int n = cls_n[c], n2 = n * n;
  const double* Vc = V + cls_V[c];
  double2* A = sm;
  double2* B = sm + n2;
  int64_t base = dof_off[e];
  for (int t = threadIdx.x; t < n2; t += NT) A[t] = X[(base + t) * R + r];
  __syncthreads();
  for (int t = threadIdx.x; t < n2; t += NT) {
    int i = t % n, j = t / n;
    double ax = 0, ay = 0;
    for (int a = 0; a < n; ++a) {
      double v = Vc[i + n * a];
      ax += v * A[a + n * j].x;
      ay += v * A[a + n * j].y;
    }
    B[t] = make_double2(ax, ay);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n2; t += NT) {
    int i = t % n, j = t / n;
    double ax = 0, ay = 0;
    for (int b = 0; b < n; ++b) {
      double v = Vc[j + n * b];
      ax += v * B[i + n * b].x;
      ay += v * B[i + n * b].y;
    }
    field[(int64_t)r * rhs_stride + base + t] = make_double2(ax, ay);
  }
}

// ---------------------------------------------------------------------------
// Krylov kernels.  R divides NT; thread t owns RHS column t % R.
__global__ void __launch_bounds__(NT) k_dots(const double2* __restrict__ V, int64_t vstride, int nvec,
                                             const double2* __restrict__ w, int n, int R,
                                             double2* __restrict__ part) {
  __shared__ double2 red[NT];
  const int r = threadIdx.x % R;
  const int rl = threadIdx.x / R;
  const int step = NT / R;
  const int64_t chunk = ((int64_t)n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = min((int64_t)n, lo + chunk);
  for (int i = 0; i < nvec; ++i) {
    const double2* Vi = V + (int64_t)i * vstride;
    double ax = 0, ay = 0;
    for (int64_t row = lo + rl; row < hi; row += step) {
      double2 a = Vi[row * R + r], b = w[row * R + r];
      ax += a.x * b.x + a.y * b.y;
      ay += a.x * b.y - a.y * b.x;
    }
    red[threadIdx.x] = make_double2(ax, ay);
    __syncthreads();
    for (int s = NT / 2; s >= R; s >>= 1) {
      if (threadIdx.x < s) {
        red[threadIdx.x].x += red[threadIdx.x + s].x;
        red[threadIdx.x].y += red[threadIdx.x + s].y;
      }
      __syncthreads();
    }
    if (threadIdx.x < R) part[((int64_t)blockIdx.x * nvec + i) * R + threadIdx.x] = red[threadIdx.x];
    __syncthreads();
  }
}

__global__ void k_dots_final(const double2* __restrict__ part, int nblk, int nvec, int R,
                             double2* __restrict__ h, double2* __restrict__ hsum) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nvec * R) return;
  double ax = 0, ay = 0;
  for (int b = 0; b < nblk; ++b) {
    double2 a = part[(int64_t)b * nvec * R + idx];
    ax += a.x;
    ay += a.y;
  }
  h[idx] = make_double2(ax, ay);
  if (hsum) {
    hsum[idx].x += ax;
    hsum[idx].y += ay;
  }
}

__global__ void k_update(const double2* __restrict__ V, int64_t vstride, int nvec,
                         const double2* __restrict__ hc, double2* __restrict__ w, int n, int R, double sign) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * R) return;
  int r = int(idx % R);
  double2 acc = w[idx];
  for (int i = 0; i < nvec; ++i) {
    double2 p = cmul(V[(int64_t)i * vstride + idx], hc[i * R + r]);
    acc.x += sign * p.x;
    acc.y += sign * p.y;
  }
  w[idx] = acc;
}

__global__ void __launch_bounds__(NT) k_norm_part(const double2* __restrict__ w, int n, int R,
                                                  double* __restrict__ part) {
  __shared__ double red[NT];
  const int r = threadIdx.x % R;
  const int rl = threadIdx.x / R;
  const int rows_per_pass = NT / R;
  double acc = 0;
  for (int64_t row = (int64_t)blockIdx.x * rows_per_pass + rl; row < n; row += (int64_t)gridDim.x * rows_per_pass) {
    double2 a = w[row * R + r];
    acc += a.x * a.x + a.y * a.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = NT / 2; s >= R; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < R) part[blockIdx.x * R + threadIdx.x] = red[threadIdx.x];
}

__global__ void k_norm_final(const double* __restrict__ part, int nblk, int R, double* __restrict__ nrm) {
  int r = threadIdx.x;
  if (r >= R) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[b * R + r];
  nrm[r] = sqrt(s);
}

__global__ void k_scale(const double2* __restrict__ w, const double* __restrict__ nrm, double2* __restrict__ out,
                        int n, int R) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * R) return;
  double d = nrm[idx % R];
  double s = d > 0 ? 1.0 / d : 0.0;
  out[idx] = make_double2(w[idx].x * s, w[idx].y * s);
}

__global__ void k_axpby(const double2* __restrict__ x, const double2* __restrict__ y, double2* __restrict__ z,
                        int64_t count, double a, double b) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  double2 p = x[idx], q = y ? y[idx] : make_double2(0, 0);
  z[idx] = make_double2(a * p.x + b * q.x, a * p.y + b * q.y);
}

__global__ void k_cast_f(const double2* __restrict__ x, float2* __restrict__ y, int64_t count) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) y[idx] = make_float2(float(x[idx].x), float(x[idx].y));
}
__global__ void k_cast_d(const float2* __restrict__ x, double2* __restrict__ y, int64_t count) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) y[idx] = make_double2(double(x[idx].x), double(x[idx].y));
}

__global__ void k_dense_scatter(const int64_t* __restrict__ idx, const double2* __restrict__ val, int64_t nnz,
                                double2* __restrict__ M) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nnz) M[idx[t]] = val[t];
}

inline unsigned nblocks(int64_t n, int t = NT) { return unsigned((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------------------
template <class T2>
void launch_slot_apply(const Handle& h, int mode, const T2* v, T2* X, T2* GL, int R, hipStream_t s) {
  dim3 grid(h.E, (R + RC - 1) / RC);
  const auto& d = h.d;
  const T2* op1;
  const typename Scal<T2>::T* se;
  if constexpr (std::is_same<T2, double2>::value) { op1 = d.op1; se = d.se; }
  else { op1 = d.op1_f; se = d.se_f; }
  if (mode == 0)
    hipLaunchKernelGGL((k_slot_apply<T2, 0>), grid, dim3(NT), 0, s, d.order, d.elem_cls, d.slot_off, d.cm_off,
                       d.cls_m, d.cls_nr, d.cls_op1, op1, se, d.cls_se, d.slot_row, d.slot_coef, d.row_xinv, v, X,
                       GL, R);
  else
    hipLaunchKernelGGL((k_slot_apply<T2, 1>), grid, dim3(NT), 0, s, d.order, d.elem_cls, d.slot_off, d.cm_off,
                       d.cls_m, d.cls_nr, d.cls_op1, op1, se, d.cls_se, d.slot_row, d.slot_coef, d.row_xinv, v, X,
                       GL, R);
  HIPCHECK(hipGetLastError());
}

template <class T2>
void launch_slot_coarse(const Handle& h, const T2* X, const double2* w, T2* Z, int R, hipStream_t s) {
  dim3 grid(h.E, (R + RC - 1) / RC);
  const auto& d = h.d;
  const T2* phi;
  if constexpr (std::is_same<T2, double2>::value) phi = d.phi; else phi = d.phi_f;
  hipLaunchKernelGGL((k_slot_coarse<T2>), grid, dim3(NT), 0, s, d.order, d.elem_cls, d.slot_off, d.cm_off, d.cls_m,
                     d.cls_nr, d.cls_phi, phi, d.cm_dof, X, w, Z, R);
  HIPCHECK(hipGetLastError());
}

template <class T2>
void launch_rowgather(const Handle& h, const T2* src, bool full, bool precond, double2* u, int R, hipStream_t s) {
  const auto& d = h.d;
  hipLaunchKernelGGL((k_rowgather<T2>), dim3(nblocks(int64_t(h.nlam) * R)), dim3(NT), 0, s, h.nlam, d.row_slot,
                     d.row_coef, precond ? d.row_xinv : nullptr, full ? d.slot_pos : nullptr, src, u, R);
  HIPCHECK(hipGetLastError());
}

template <class T2>
void launch_assemble(const Handle& h, const T2* GL, const double2* Bfull, double2* g, int R, hipStream_t s) {
  const auto& d = h.d;
  hipLaunchKernelGGL((k_assemble<T2>), dim3(nblocks(int64_t(h.nK) * R)), dim3(NT), 0, s, h.nK, d.cdof_ptr,
                     d.cdof_list, GL, d.cm_pos, Bfull, g, R);
  HIPCHECK(hipGetLastError());
}

template void launch_slot_apply<double2>(const Handle&, int, const double2*, double2*, double2*, int, hipStream_t);
template void launch_slot_apply<float2>(const Handle&, int, const float2*, float2*, float2*, int, hipStream_t);
template void launch_slot_coarse<double2>(const Handle&, const double2*, const double2*, double2*, int, hipStream_t);
template void launch_slot_coarse<float2>(const Handle&, const float2*, const double2*, float2*, int, hipStream_t);
template void launch_rowgather<double2>(const Handle&, const double2*, bool, bool, double2*, int, hipStream_t);
template void launch_rowgather<float2>(const Handle&, const float2*, bool, bool, double2*, int, hipStream_t);
template void launch_assemble<double2>(const Handle&, const double2*, const double2*, double2*, int, hipStream_t);
template void launch_assemble<float2>(const Handle&, const float2*, const double2*, double2*, int, hipStream_t);

void launch_coarse_solve(const Handle& h, const double2* g, double2* w, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_gemv, dim3(nblocks(h.nK, NT / 64)), dim3(NT), 0, s, h.nK, h.d.Kinv, g, w, R);
  HIPCHECK(hipGetLastError());
}

void launch_fdm(const Handle& h, const double2* in, double2* out, int R, hipStream_t s) {
  int nmax = 0;
  for (auto& C : h.classes) nmax = std::max(nmax, C.n);
  size_t shm = size_t(2) * nmax * nmax * sizeof(double2);
  const auto& d = h.d;
  hipLaunchKernelGGL(k_fdm, dim3(h.E, R), dim3(NT), shm, s, d.elem_cls, d.dof_off, d.cls_n, d.cls_E, d.cls_D, d.Ex,
                     d.Ey, d.Dinv, in, out, R);
  HIPCHECK(hipGetLastError());
}

void launch_zero_R(const Handle& h, double2* X, int R, hipStream_t s) {
  const auto& d = h.d;
  hipLaunchKernelGGL(k_zero_R, dim3(h.E), dim3(64), 0, s, h.E, d.elem_cls, d.dof_off, d.cls_nr, d.cls_R, d.r_modes,
                     X, R);
  HIPCHECK(hipGetLastError());
}

void launch_extract_kc(const Handle& h, const double2* X, double2* GL, int R, hipStream_t s) {
  const auto& d = h.d;
  hipLaunchKernelGGL(k_extract_kc, dim3(h.E, R), dim3(64), 0, s, d.elem_cls, d.dof_off, d.cm_off, d.cls_nr, d.cls_R,
                     d.r_modes, d.cls_Kc, d.Kc, X, GL, R);
  HIPCHECK(hipGetLastError());
}

void launch_correct(const Handle& h, double2* X, const double2* w, int R, hipStream_t s) {
  const auto& d = h.d;
  hipLaunchKernelGGL(k_correct, dim3(h.E, R), dim3(NT), 0, s, d.elem_cls, d.dof_off, d.cm_off, d.cls_n, d.cls_nr,
                     d.cls_R, d.r_modes, d.cls_Kc, d.Kc, d.cls_G, d.G, d.cm_dof, X, w, R);
  HIPCHECK(hipGetLastError());
}

void launch_sub_dual(const Handle& h, double2* Y, const double2* nu, int R, hipStream_t s) {
  const auto& d = h.d;
  hipLaunchKernelGGL(k_sub_dual, dim3(nblocks(int64_t(h.nslots) * R)), dim3(NT), 0, s, h.nslots, d.slot_pos,
                     d.slot_row, d.slot_coef, Y, nu, R);
  HIPCHECK(hipGetLastError());
}

void launch_gll(const Handle& h, const double2* X, double2* field, int R, int64_t rhs_stride, int nrhs_out,
                hipStream_t s) {
  int nmax = 0;
  for (auto& C : h.classes) nmax = std::max(nmax, C.n);
  size_t shm = size_t(2) * nmax * nmax * sizeof(double2);
  const auto& d = h.d;
  hipLaunchKernelGGL(k_gll, dim3(h.E, nrhs_out), dim3(NT), shm, s, d.elem_cls, d.dof_off, d.cls_n, d.cls_V, d.V, X,
                     field, R, rhs_stride);
  HIPCHECK(hipGetLastError());
}

int dots_blocks(int n, int R) {
  int64_t want = (int64_t(n) * R + NT - 1) / NT;
  return int(std::max<int64_t>(1, std::min<int64_t>(512, want)));
}

void launch_dots(const double2* V, int64_t vstride, int nvec, const double2* w, int n, int R, double2* part, int nblk,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3(nblk), dim3(NT), 0, s, V, vstride, nvec, w, n, R, part);
  HIPCHECK(hipGetLastError());
}

void launch_dots_final(const double2* part, int nblk, int nvec, int R, double2* hh, double2* hsum, hipStream_t s) {
  hipLaunchKernelGGL(k_dots_final, dim3(nblocks(int64_t(nvec) * R)), dim3(NT), 0, s, part, nblk, nvec, R, hh, hsum);
  HIPCHECK(hipGetLastError());
}

void launch_update(const double2* V, int64_t vstride, int nvec, const double2* hc, double2* w, int n, int R,
                   double sign, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(nblocks(int64_t(n) * R)), dim3(NT), 0, s, V, vstride, nvec, hc, w, n, R, sign);
  HIPCHECK(hipGetLastError());
}

void launch_norm(const double2* w, int n, int R, double* part, int nblk, double* nrm, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_part, dim3(nblk), dim3(NT), 0, s, w, n, R, part);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(NT), 0, s, part, nblk, R, nrm);
  HIPCHECK(hipGetLastError());
}

void launch_scale(const double2* w, const double* nrm, double2* out, int n, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(nblocks(int64_t(n) * R)), dim3(NT), 0, s, w, nrm, out, n, R);
  HIPCHECK(hipGetLastError());
}

void launch_axpby(const double2* x, const double2* y, double2* z, int64_t count, double a, double b, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(nblocks(count)), dim3(NT), 0, s, x, y, z, count, a, b);
  HIPCHECK(hipGetLastError());
}

void launch_cast_f(const double2* x, float2* y, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f, dim3(nblocks(count)), dim3(NT), 0, s, x, y, count);
  HIPCHECK(hipGetLastError());
}

void launch_cast_d(const float2* x, double2* y, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_d, dim3(nblocks(count)), dim3(NT), 0, s, x, y, count);
  HIPCHECK(hipGetLastError());
}

void launch_dense_scatter(const int64_t* idx, const double2* val, int64_t nnz, double2* M, hipStream_t s) {
  if (nnz == 0) return;
  hipLaunchKernelGGL(k_dense_scatter, dim3(nblocks(nnz)), dim3(NT), 0, s, idx, val, nnz, M);
  HIPCHECK(hipGetLastError());
}

}  // namespace hdp
