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

// Reduce a per-thread value over the threads of a block that share an RHS
// column (lanes with equal lane % R inside a wave, then the four waves).
__device__ __forceinline__ double2 block_sum_by_rhs(double2 v, int R, double2* red) {
  for (int off = 32; off >= R && off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane < R) red[wv * 64 + lane] = v;
  __syncthreads();
  double2 s = make_double2(0, 0);
  if (threadIdx.x < R)
    for (int q = 0; q < NT / 64; ++q) {
      s.x += red[q * 64 + threadIdx.x].x;
      s.y += red[q * 64 + threadIdx.x].y;
    }
  __syncthreads();
  return s;   // valid in threads 0..R-1
}

// ---------------------------------------------------------------------------
// Slot kernels: one block per element (class-grouped order), RC RHS per block.
template <class T2, int MODE>
__global__ void __launch_bounds__(NT) k_slot_apply(const SlotBlock* __restrict__ blk, const SlotIn* __restrict__ sin,
                                                   const T2* __restrict__ op1, const T2* __restrict__ se,
                                                   const T2* __restrict__ v, T2* __restrict__ X, T2* __restrict__ GL,
                                                   int R) {
  using S = typename Scal<T2>::T;
  __shared__ T2 y[MMAX * RC];
  const SlotBlock B = blk[blockIdx.x];
  const int m = B.m, nr = B.nr, so = B.so;
  const int r0 = blockIdx.y * RC;
  const int rc = min(RC, R - r0);
  for (int idx = threadIdx.x; idx < m * rc; idx += NT) {
    const int s = idx / rc, r = idx - s * rc;
    // MODE 0/1: v holds dual rows; MODE 2: dual slots, the row value being the
    // jump C_1 z of its two slots
    const SlotIn g = sin[so + s];
    S ax = 0, ay = 0;
    if (g.s0 >= 0) {
      const T2 z = v[(int64_t)g.s0 * R + r0 + r];
      ax += S(g.a0) * z.x;
      ay += S(g.a0) * z.y;
    }
    if (MODE == 2 && g.s1 >= 0) {
      const T2 z = v[(int64_t)g.s1 * R + r0 + r];
      ax += S(g.a1) * z.x;
      ay += S(g.a1) * z.y;
    }
    y[s * RC + r] = mk<T2>(ax, ay);
  }
  __syncthreads();
  if (MODE == 0) {
    const int nrow = m + nr;
    const T2* A = op1 + B.op1;
    for (int idx = threadIdx.x; idx < nrow * rc; idx += NT) {
      int i = idx / rc, r = idx - i * rc;
      T2 acc = mk<T2>(0, 0);
      for (int kk = 0; kk < m; ++kk) acc = cfma(A[i + (int64_t)nrow * kk], y[kk * RC + r], acc);
      if (i < m) X[(int64_t)(so + i) * R + r0 + r] = acc;
      else GL[(int64_t)(B.cmo + i - m) * R + r0 + r] = acc;
    }
  } else {
    const T2* A = se + B.se;
    for (int idx = threadIdx.x; idx < m * rc; idx += NT) {
      int i = idx / rc, r = idx - i * rc;
      T2 acc = mk<T2>(0, 0);
      for (int kk = 0; kk < m; ++kk) acc = cfma(A[i + (int64_t)m * kk], y[kk * RC + r], acc);
      X[(int64_t)(so + i) * R + r0 + r] = acc;
    }
  }
}

// The preconditioner on dual slots (S_e on the jumps C_1 z of each element's
// slots) with the row gather fused: every output slot adds its value times its
// row coefficient into the dual row.  A row has at most two slots and out is
// zero on entry, so the two additions give the same sum in either order.
__global__ void __launch_bounds__(NT) k_slot_apply_rows(const SlotBlock* __restrict__ blk,
                                                        const SlotIn* __restrict__ sin,
                                                        const SlotOut* __restrict__ sout,
                                                        const double2* __restrict__ se,
                                                        const double2* __restrict__ v, double2* __restrict__ out,
                                                        int R) {
  __shared__ double2 y[MMAX * RC];
  const SlotBlock B = blk[blockIdx.x];
  const int m = B.m, so = B.so;
  const int r0 = blockIdx.y * RC;
  const int rc = min(RC, R - r0);
  for (int idx = threadIdx.x; idx < m * rc; idx += NT) {
    const int sl = idx / rc, r = idx - sl * rc;
    const SlotIn g = sin[so + sl];
    double ax = 0, ay = 0;
    if (g.s0 >= 0) {
      const double2 z = v[(int64_t)g.s0 * R + r0 + r];
      ax += g.a0 * z.x;
      ay += g.a0 * z.y;
    }
    if (g.s1 >= 0) {
      const double2 z = v[(int64_t)g.s1 * R + r0 + r];
      ax += g.a1 * z.x;
      ay += g.a1 * z.y;
    }
    y[sl * RC + r] = make_double2(ax, ay);
  }
  __syncthreads();
  const double2* A = se + B.se;
  for (int idx = threadIdx.x; idx < m * rc; idx += NT) {
    const int i = idx / rc, r = idx - i * rc;
    double2 acc = make_double2(0, 0);
    for (int kk = 0; kk < m; ++kk) acc = cfma(A[i + (int64_t)m * kk], y[kk * RC + r], acc);
    const SlotOut o = sout[so + i];
    double2* p = out + (int64_t)o.row * R + r0 + r;
    unsafeAtomicAdd(&p->x, o.coef * acc.x);
    unsafeAtomicAdd(&p->y, o.coef * acc.y);
  }
}

template <class T2>
__global__ void __launch_bounds__(NT) k_slot_coarse(const SlotBlock* __restrict__ blk, const T2* __restrict__ phi,
                                                    const int* __restrict__ t_ptr, const int* __restrict__ t_dof,
                                                    const double* __restrict__ t_coef, const T2* __restrict__ X,
                                                    const double2* __restrict__ w, T2* __restrict__ Z, int R) {
  __shared__ T2 we[NRMAX * RC];
  const SlotBlock B = blk[blockIdx.x];
  const int m = B.m, nr = B.nr, co = B.cmo, so = B.so;
  const int r0 = blockIdx.y * RC;
  const int rc = min(RC, R - r0);
  if (rc == 1) {
    // one column: each coarse mode's expansion (long on hanging edges) is split
    // over RC threads whose partial sums sit in we[j RC .. j RC + RC) and are
    // added in order into we[j RC]
    for (int idx = threadIdx.x; idx < nr * RC; idx += NT) {
      const int j = idx / RC, q = idx - j * RC;
      double ax = 0, ay = 0;
      for (int t = t_ptr[co + j] + q; t < t_ptr[co + j + 1]; t += RC) {
        const double2 a = w[(int64_t)t_dof[t] * R + r0];
        ax += t_coef[t] * a.x;
        ay += t_coef[t] * a.y;
      }
      we[idx] = mk<T2>(ax, ay);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nr; j += NT) {
      T2 sum = we[j * RC];
      for (int q = 1; q < RC; ++q) {
        const T2 p = we[j * RC + q];
        sum.x += p.x;
        sum.y += p.y;
      }
      we[j * RC] = sum;
    }
  } else {
    for (int idx = threadIdx.x; idx < nr * rc; idx += NT) {
      int j = idx / rc, r = idx - j * rc;
      double ax = 0, ay = 0;
      for (int t = t_ptr[co + j]; t < t_ptr[co + j + 1]; ++t) {
        double2 a = w[(int64_t)t_dof[t] * R + r0 + r];
        ax += t_coef[t] * a.x;
        ay += t_coef[t] * a.y;
      }
      we[j * RC + r] = mk<T2>(ax, ay);
    }
  }
  __syncthreads();
  const T2* P = phi + B.phi;
  for (int idx = threadIdx.x; idx < m * rc; idx += NT) {
    int i = idx / rc, r = idx - i * rc;
    T2 acc = X[(int64_t)(so + i) * R + r0 + r];
    for (int j = 0; j < nr; ++j) acc = cfma(P[i + (int64_t)m * j], we[j * RC + r], acc);
    Z[(int64_t)(so + i) * R + r0 + r] = acc;
  }
}

typedef double d4 __attribute__((ext_vector_type(4)));

// The slot operators at 16, 32 or 64 right-hand sides on the FP64 matrix
// cores.  Per element (block): the K x R operand (gathered dual slots, or the
// element's coarse values for MODE 3) goes to LDS with R fastest; out = Mat
// operand, Mat column-major nrow x K (op1 for MODE 0, S_e for MODEs 1/2, Phi for
// MODE 3, which also adds X).  Wave w owns output tiles (16 rows of Mat) x (16
// columns of R) in turn; a step of 4 summation rows is four real 16x16x4
// operations per complex tile (A operand: 16 columns of R x 4 rows from LDS, B
// operand: 4 rows x 16 rows of Mat).  Lane l holds result (column (l >> 4) + 4 v,
// row l & 15) in value v; the tiles are written back to the LDS buffer and
// copied out with R fastest.  The LDS buffer holds max(K, nrow) x R entries
// (at most the largest such count over the classes, times R).
constexpr int SLOT_MF_LDS = 65536;
constexpr int SLOT_GB = 4;   // gathered operand entries per thread and pass

// The coarse values (T_e w)[kk][r] of an element's coarse modes kk < K (their
// expansions over the coarse unknowns, from t_ptr[cmo + kk]) for the RB columns
// from r0, into out (K x RB, r fastest).  SLOT_GB entries per thread and pass:
// the first term of every expansion (pointer, then index and coefficient, then
// the row of w) is requested for all of them before any is used; further terms
// (modes on hanging edges) follow in expansion order.
template <class OT>
__device__ __forceinline__ void gather_coarse(const int* __restrict__ t_ptr, const int* __restrict__ t_dof,
                                              const double* __restrict__ t_coef, const double2* __restrict__ v,
                                              int cmo, int K, int RB, int R, int r0, OT* out) {
  for (int i0 = threadIdx.x; i0 < K * RB; i0 += NT * SLOT_GB) {
    int p0[SLOT_GB], p1[SLOT_GB];
#pragma unroll
    for (int u = 0; u < SLOT_GB; ++u) {
      const int co = cmo + min(i0 + u * NT, K * RB - 1) / RB;
      p0[u] = t_ptr[co];
      p1[u] = t_ptr[co + 1];
    }
    int d[SLOT_GB];
    double c[SLOT_GB];
#pragma unroll
    for (int u = 0; u < SLOT_GB; ++u) {
      const bool has = p1[u] > p0[u];
      d[u] = has ? t_dof[p0[u]] : -1;
      c[u] = has ? t_coef[p0[u]] : 0.0;
    }
    double2 z[SLOT_GB];
#pragma unroll
    for (int u = 0; u < SLOT_GB; ++u) {
      const int idx = i0 + u * NT, r = idx % RB;
      z[u] = make_double2(0, 0);
      if (idx < K * RB && d[u] >= 0) z[u] = v[(int64_t)d[u] * R + r0 + r];
    }
#pragma unroll
    for (int u = 0; u < SLOT_GB; ++u) {
      const int idx = i0 + u * NT, r = idx % RB;
      if (idx >= K * RB) break;
      double sx = c[u] * z[u].x, sy = c[u] * z[u].y;
      for (int t = p0[u] + 1; t < p1[u]; ++t) {
        const double2 a = v[(int64_t)t_dof[t] * R + r0 + r];
        sx += t_coef[t] * a.x;
        sy += t_coef[t] * a.y;
      }
      out[idx] = mk<OT>(sx, sy);
    }
  }
}

// (at most 128 registers: four blocks per compute unit where the shared memory
// allows them; unbounded the compiler took 146 and three)
template <int MODE>
__global__ void __launch_bounds__(NT, 4) k_slot_mfma(const SlotBlock* __restrict__ blk,
                                                  const SlotIn* __restrict__ sin, const double2* __restrict__ op1,
                                                  const double2* __restrict__ se, const double2* __restrict__ phi,
                                                  const int* __restrict__ t_ptr, const int* __restrict__ t_dof,
                                                  const double* __restrict__ t_coef, const double2* __restrict__ v,
                                                  const double2* __restrict__ Xin, double2* __restrict__ X,
                                                  double2* __restrict__ GL, int R, int RB) {
  extern __shared__ double2 buf[];
  const int r0 = blockIdx.y * RB;   // this block's RB columns of the R
  const SlotBlock B = blk[blockIdx.x];
  const int m = B.m, nr = B.nr, so = B.so;
  const int K = MODE == 3 ? nr : m;
  const int nrow = MODE == 0 ? m + nr : m;
  const double2* Mat = MODE == 0 ? op1 + B.op1 : (MODE == 3 ? phi + B.phi : se + B.se);
  // operand rows kk x R
  if (MODE == 3) {
    gather_coarse<double2>(t_ptr, t_dof, t_coef, v, B.cmo, K, RB, R, r0, buf);
  } else {
    // SLOT_GB entries per thread and pass: the slot records, then the gathered
    // rows, are all requested before any is used
    for (int i0 = threadIdx.x; i0 < K * RB; i0 += NT * SLOT_GB) {
      SlotIn g[SLOT_GB];
#pragma unroll
      for (int u = 0; u < SLOT_GB; ++u) {
        const int idx = min(i0 + u * NT, K * RB - 1);
        g[u] = sin[so + idx / RB];
      }
      double2 z0[SLOT_GB], z1[SLOT_GB];
#pragma unroll
      for (int u = 0; u < SLOT_GB; ++u) {
        const int idx = i0 + u * NT, r = idx % RB;
        z0[u] = z1[u] = make_double2(0, 0);
        if (idx < K * RB && g[u].s0 >= 0) z0[u] = v[(int64_t)g[u].s0 * R + r0 + r];
        if (MODE == 2 && idx < K * RB && g[u].s1 >= 0) z1[u] = v[(int64_t)g[u].s1 * R + r0 + r];
      }
#pragma unroll
      for (int u = 0; u < SLOT_GB; ++u) {
        const int idx = i0 + u * NT;
        if (idx >= K * RB) break;
        double ax = g[u].a0 * z0[u].x, ay = g[u].a0 * z0[u].y;
        if (MODE == 2) {
          ax += g[u].a1 * z1[u].x;
          ay += g[u].a1 * z1[u].y;
        }
        buf[idx] = make_double2(ax, ay);
      }
    }
  }
  __syncthreads();
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jl = l & 15, kq = l >> 4;
  const int nit = (nrow + 15) >> 4, nrt = RB >> 4, ntile = nit * nrt;
  // at most 4 row tiles x 4 column tiles: each wave keeps up to 4 tiles
  d4 cr[4], ci[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cr[q] = (d4){0, 0, 0, 0};
    ci[q] = (d4){0, 0, 0, 0};
  }
  // two steps of 4 summation rows per pass: the operator entries of both steps
  // (global, cached) are requested before their matrix operations (one step per
  // pass for MODE 3, whose gather of coarse values needs the occupancy more)
  constexpr int NS = MODE == 3 ? 1 : 2;
  for (int k0 = 0; k0 < K; k0 += 4 * NS) {
    double2 bq[NS][4];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int kk = k0 + 4 * st + kq;
      const bool kv = kk < K;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tile = min(wv + 4 * q, ntile - 1);
        const int it = tile / nrt;
        const int i = 16 * it + jl;
        bq[st][q] = (kv && i < nrow) ? Mat[i + (int64_t)nrow * kk] : make_double2(0, 0);
      }
    }
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int kk = k0 + 4 * st + kq;
      const bool kv = kk < K;
      if (k0 + 4 * st >= K) break;   // uniform: a step wholly past K
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tile = wv + 4 * q;
        if (tile >= ntile) break;   // uniform over the wave
        const int rt = tile - (tile / nrt) * nrt;
        const double2 b = bq[st][q];
        const double2 a = kv ? buf[kk * RB + 16 * rt + jl] : make_double2(0, 0);
        cr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr[q], 0, 0, 0);
        ci[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci[q], 0, 0, 0);
        cr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr[q], 0, 0, 0);
        ci[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci[q], 0, 0, 0);
      }
    }
  }
  __syncthreads();   // every wave is done with the operand
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int tile = wv + 4 * q;
    if (tile >= ntile) break;
    const int it = tile / nrt, rt = tile - it * nrt;
    const int i = 16 * it + jl;
    if (i < nrow) {
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) buf[i * RB + 16 * rt + kq + 4 * vv] = make_double2(cr[q][vv], ci[q][vv]);
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nrow * RB; idx += NT) {
    const int i = idx / RB, r = idx - i * RB;
    double2 o = buf[idx];
    if (MODE == 3) {
      const double2 x = Xin[(int64_t)(so + i) * R + r0 + r];
      o.x += x.x;
      o.y += x.y;
    }
    if (MODE != 0 || i < m) X[(int64_t)(so + i) * R + r0 + r] = o;
    else GL[(int64_t)(B.cmo + i - m) * R + r0 + r] = o;
  }
}

typedef float f4 __attribute__((ext_vector_type(4)));

// The slot operators of the mixed-precision path at 16, 32 or 64 right-hand
// sides on the FP32 matrix cores (FP32 operators and operands, FP32
// accumulation), laid out as k_slot_mfma: the K x RB operand in shared memory
// with R fastest, out = Mat operand, a step of 4 summation rows as four real
// 16x16x4 FP32 operations per complex tile.  The FP32 operation returns, in lane
// l and value v, row 4 (l >> 4) + v (the operand column) and column l & 15 (the
// row of Mat) of its 16 x 16 tile.  VT is the operand source type: FP32 dual or
// slot values, or (MODE 3) the FP64 coarse solution gathered through T.
template <int MODE, class VT>
__global__ void __launch_bounds__(NT) k_slot_mfma32(const SlotBlock* __restrict__ blk,
                                                    const SlotIn* __restrict__ sin, const float2* __restrict__ op1,
                                                    const float2* __restrict__ se, const float2* __restrict__ phi,
                                                    const int* __restrict__ t_ptr, const int* __restrict__ t_dof,
                                                    const double* __restrict__ t_coef, const VT* __restrict__ v,
                                                    const float2* __restrict__ Xin, float2* __restrict__ X,
                                                    float2* __restrict__ GL, int R, int RB) {
  extern __shared__ float2 buf32[];
  const int r0 = blockIdx.y * RB;
  const SlotBlock B = blk[blockIdx.x];
  const int m = B.m, nr = B.nr, so = B.so;
  const int K = MODE == 3 ? nr : m;
  const int nrow = MODE == 0 ? m + nr : m;
  const float2* Mat = MODE == 0 ? op1 + B.op1 : (MODE == 3 ? phi + B.phi : se + B.se);
  if (MODE == 3) {
    if constexpr (std::is_same<VT, double2>::value) gather_coarse<float2>(t_ptr, t_dof, t_coef, v, B.cmo, K, RB, R, r0, buf32);
  } else {
    // as k_slot_mfma: the slot records, then the gathered rows, all requested
    // before any is used
    for (int i0 = threadIdx.x; i0 < K * RB; i0 += NT * SLOT_GB) {
      SlotIn g[SLOT_GB];
#pragma unroll
      for (int u = 0; u < SLOT_GB; ++u) {
        const int idx = min(i0 + u * NT, K * RB - 1);
        g[u] = sin[so + idx / RB];
      }
      VT z0[SLOT_GB], z1[SLOT_GB];
#pragma unroll
      for (int u = 0; u < SLOT_GB; ++u) {
        const int idx = i0 + u * NT, r = idx % RB;
        z0[u].x = z0[u].y = z1[u].x = z1[u].y = 0;
        if (idx < K * RB && g[u].s0 >= 0) z0[u] = v[(int64_t)g[u].s0 * R + r0 + r];
        if (MODE == 2 && idx < K * RB && g[u].s1 >= 0) z1[u] = v[(int64_t)g[u].s1 * R + r0 + r];
      }
#pragma unroll
      for (int u = 0; u < SLOT_GB; ++u) {
        const int idx = i0 + u * NT;
        if (idx >= K * RB) break;
        float ax = float(g[u].a0) * z0[u].x, ay = float(g[u].a0) * z0[u].y;
        if (MODE == 2) {
          ax += float(g[u].a1) * z1[u].x;
          ay += float(g[u].a1) * z1[u].y;
        }
        buf32[idx] = make_float2(ax, ay);
      }
    }
  }
  __syncthreads();
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jl = l & 15, kq = l >> 4;
  const int nit = (nrow + 15) >> 4, nrt = RB >> 4, ntile = nit * nrt;
  f4 cr[4], ci[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cr[q] = (f4){0, 0, 0, 0};
    ci[q] = (f4){0, 0, 0, 0};
  }
  constexpr int NS = MODE == 3 ? 1 : 2;   // steps per pass, operator loads first (as k_slot_mfma)
  for (int k0 = 0; k0 < K; k0 += 4 * NS) {
    float2 bq[NS][4];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int kk = k0 + 4 * st + kq;
      const bool kv = kk < K;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tile = min(wv + 4 * q, ntile - 1);
        const int i = 16 * (tile / nrt) + jl;
        bq[st][q] = (kv && i < nrow) ? Mat[i + (int64_t)nrow * kk] : make_float2(0, 0);
      }
    }
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int kk = k0 + 4 * st + kq;
      const bool kv = kk < K;
      if (k0 + 4 * st >= K) break;   // uniform: a step wholly past K
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tile = wv + 4 * q;
        if (tile >= ntile) break;   // uniform over the wave
        const int rt = tile - (tile / nrt) * nrt;
        const float2 b = bq[st][q];
        const float2 a = kv ? buf32[kk * RB + 16 * rt + jl] : make_float2(0, 0);
        cr[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cr[q], 0, 0, 0);
        ci[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, ci[q], 0, 0, 0);
        cr[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, cr[q], 0, 0, 0);
        ci[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, ci[q], 0, 0, 0);
      }
    }
  }
  __syncthreads();   // every wave is done with the operand
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int tile = wv + 4 * q;
    if (tile >= ntile) break;
    const int it = tile / nrt, rt = tile - it * nrt;
    const int i = 16 * it + jl;
    if (i < nrow) {
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) buf32[i * RB + 16 * rt + 4 * kq + vv] = make_float2(cr[q][vv], ci[q][vv]);
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nrow * RB; idx += NT) {
    const int i = idx / RB, r = idx - i * RB;
    float2 o = buf32[idx];
    if (MODE == 3) {
      const float2 x = Xin[(int64_t)(so + i) * R + r0 + r];
      o.x += x.x;
      o.y += x.y;
    }
    if (MODE != 0 || i < m) X[(int64_t)(so + i) * R + r0 + r] = o;
    else GL[(int64_t)(B.cmo + i - m) * R + r0 + r] = o;
  }
}

// k_slot_coarse with the coarse solution taken straight from the partial sums
// of the tiled coarse apply (one right-hand side): w[d] = sum_J P[d / 64][J][d % 64],
// each coarse mode's sum split over SCP thread groups and added in a fixed
// order, so the row-sum kernel is not needed.
constexpr int SCP = 16;
constexpr int SYM_TILE = 64;   // tile edge of the symmetric coarse inverse

template <class T2>
__global__ void __launch_bounds__(NT) k_slot_coarse_sym(const SlotBlock* __restrict__ blk, const T2* __restrict__ phi,
                                                        const int* __restrict__ t_ptr, const int* __restrict__ t_dof,
                                                        const double* __restrict__ t_coef,
                                                        const T2* __restrict__ X, const double2* __restrict__ P,
                                                        int nt, T2* __restrict__ Z) {
  extern __shared__ double2 part[];   // nr x SCP partial sums of the largest class
  __shared__ T2 we[NRMAX];
  const SlotBlock B = blk[blockIdx.x];
  const int m = B.m, nr = B.nr, co = B.cmo, so = B.so;
  for (int idx = threadIdx.x; idx < nr * SCP; idx += NT) {
    const int j = idx / SCP, q = idx - j * SCP;
    double ax = 0, ay = 0;
    for (int t = t_ptr[co + j]; t < t_ptr[co + j + 1]; ++t) {
      const int dof = t_dof[t];
      const double2* Pr = P + (int64_t)(dof / SYM_TILE) * nt * SYM_TILE + dof % SYM_TILE;
      double sx = 0, sy = 0;
      for (int J = q; J < nt; J += SCP) {
        const double2 a = Pr[(int64_t)J * SYM_TILE];
        sx += a.x;
        sy += a.y;
      }
      ax += t_coef[t] * sx;
      ay += t_coef[t] * sy;
    }
    part[idx] = make_double2(ax, ay);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nr; j += NT) {
    double ax = 0, ay = 0;
    for (int q = 0; q < SCP; ++q) {
      ax += part[j * SCP + q].x;
      ay += part[j * SCP + q].y;
    }
    we[j] = mk<T2>(ax, ay);
  }
  __syncthreads();
  const T2* Pm = phi + B.phi;
  for (int i = threadIdx.x; i < m; i += NT) {
    T2 acc = X[so + i];
    for (int j = 0; j < nr; ++j) acc = cfma(Pm[i + (int64_t)m * j], we[j], acc);
    Z[so + i] = acc;
  }
}

// u[row] = scale_row * (sum coef * src[pos(slot)] + sum_{C_2} coef * w[dof])
template <class T2>
__global__ void k_rowgather(int nlam, const int* __restrict__ row_slot, const double* __restrict__ row_coef,
                            const double* __restrict__ row_xinv, const int64_t* __restrict__ slot_pos,
                            const T2* __restrict__ src, const int* __restrict__ c2_ptr,
                            const int* __restrict__ c2_dof, const double* __restrict__ c2_coef,
                            const double2* __restrict__ w, double2* __restrict__ u, int R) {
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
  if (w)
    for (int t = c2_ptr[row]; t < c2_ptr[row + 1]; ++t) {
      double2 a = w[(int64_t)c2_dof[t] * R + r];
      ax += c2_coef[t] * a.x;
      ay += c2_coef[t] * a.y;
    }
  if (row_xinv) {
    ax *= row_xinv[row];
    ay *= row_xinv[row];
  }
  u[idx] = make_double2(ax, ay);
}

// The same at one right-hand side with one wave per coarse unknown, for meshes
// with hanging edges: the lanes split the unknown's expansion and C_2 entries
// (long there) and add them with shuffles, so no lane walks a long list alone.
// (On conforming meshes the lists hold one to four entries and a thread per
// unknown is faster.)
template <class T2>
__global__ void __launch_bounds__(NT) k_assemble1(int nK, const int* __restrict__ ptr, const int* __restrict__ list,
                                                  const double* __restrict__ coef, const T2* __restrict__ GL,
                                                  const int64_t* __restrict__ cm_pos,
                                                  const double2* __restrict__ Bfull, const int* __restrict__ c2t_ptr,
                                                  const int* __restrict__ c2t_row,
                                                  const double* __restrict__ c2t_coef, const double2* __restrict__ v,
                                                  double csign, double2* __restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int d = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (d >= nK) return;
  double ax = 0, ay = 0;
  for (int t = ptr[d] + lane; t < ptr[d + 1]; t += 64) {
    const int i = list[t];
    const double c = coef[t];
    if (GL) {
      const T2 a = GL[i];
      ax += c * double(a.x);
      ay += c * double(a.y);
    }
    if (Bfull) {
      const double2 b = Bfull[cm_pos[i]];
      ax += c * b.x;
      ay += c * b.y;
    }
  }
  if (v)
    for (int t = c2t_ptr[d] + lane; t < c2t_ptr[d + 1]; t += 64) {
      const double2 a = v[c2t_row[t]];
      ax += csign * c2t_coef[t] * a.x;
      ay += csign * c2t_coef[t] * a.y;
    }
  for (int off = 32; off > 0; off >>= 1) {
    ax += __shfl_xor(ax, off, 64);
    ay += __shfl_xor(ay, off, 64);
  }
  if (lane == 0) g[d] = make_double2(ax, ay);
}

// g[d] = sum_{(i, c) in T^T} c (GL[i] + Bfull[pos(i)]) + csign sum_{(row, c) in C_2^T} c v[row]
template <class T2>
__global__ void k_assemble(int nK, const int* __restrict__ ptr, const int* __restrict__ list,
                           const double* __restrict__ coef, const T2* __restrict__ GL,
                           const int64_t* __restrict__ cm_pos, const double2* __restrict__ Bfull,
                           const int* __restrict__ c2t_ptr, const int* __restrict__ c2t_row,
                           const double* __restrict__ c2t_coef, const double2* __restrict__ v, double csign,
                           double2* __restrict__ g, int R) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nK * R) return;
  int d = int(idx / R), r = int(idx - (int64_t)d * R);
  double ax = 0, ay = 0;
  for (int t = ptr[d]; t < ptr[d + 1]; ++t) {
    int i = list[t];
    double c = coef[t];
    if (GL) {
      T2 a = GL[(int64_t)i * R + r];
      ax += c * double(a.x);
      ay += c * double(a.y);
    }
    if (Bfull) {
      double2 b = Bfull[cm_pos[i] * R + r];
      ax += c * b.x;
      ay += c * b.y;
    }
  }
  if (v)
    for (int t = c2t_ptr[d]; t < c2t_ptr[d + 1]; ++t) {
      double2 a = v[(int64_t)c2t_row[t] * R + r];
      ax += csign * c2t_coef[t] * a.x;
      ay += csign * c2t_coef[t] * a.y;
    }
  g[idx] = make_double2(ax, ay);
}

// Dense blocks over the dual rows that C_2 couples (hanging edges): one
// wavefront per block row i, RHS in chunks of 8.
//   out_i = (add ? add[row_i] : 0) + sum_j M_b[i, j] in_j
// in_j is x[row_j] (gather) or x[off_b + j] (compact); out_i goes to
// y[row_i] (scatter) or y[off_b + i] (compact).
__global__ void __launch_bounds__(NT) k_hblock(int nh, const int* __restrict__ blk, const int* __restrict__ off,
                                               const int* __restrict__ rows, const int64_t* __restrict__ moff,
                                               const double* __restrict__ M, const double2* __restrict__ x,
                                               int in_gather, const double2* __restrict__ add,
                                               double2* __restrict__ y, int out_scatter, int R) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (i >= nh) return;
  const int b = blk[i], o = off[b], nb = off[b + 1] - o, il = i - o;
  const double* Mb = M + moff[b];
  for (int r0 = 0; r0 < R; r0 += 8) {
    int rc = min(8, R - r0);
    double ax[8] = {0}, ay[8] = {0};
    for (int j = lane; j < nb; j += 64) {
      double m = Mb[il + (int64_t)nb * j];
      int64_t src = in_gather ? (int64_t)rows[o + j] : (int64_t)(o + j);
      for (int r = 0; r < rc; ++r) {
        double2 v = x[src * R + r0 + r];
        ax[r] += m * v.x;
        ay[r] += m * v.y;
      }
    }
    for (int r = 0; r < rc; ++r) {
      double sx = ax[r], sy = ay[r];
      for (int sh = 32; sh > 0; sh >>= 1) {
        sx += __shfl_down(sx, sh, 64);
        sy += __shfl_down(sy, sh, 64);
      }
      if (lane == 0) {
        if (add) {
          double2 a = add[(int64_t)rows[i] * R + r0 + r];
          sx += a.x;
          sy += a.y;
        }
        int64_t dst = out_scatter ? (int64_t)rows[i] : (int64_t)i;
        y[dst * R + r0 + r] = make_double2(sx, sy);
      }
    }
  }
}

// Tiles of the nested-dissection products (several columns).
constexpr int SMJ = 32;   // outputs per workgroup
constexpr int SMK = 32;   // rows of M staged per pass

// ---------------------------------------------------------------------------
// Nested-dissection coarse solve.  Node t owns the coarse unknowns
// [off_t, off_t + nI_t) and has the boundary list bnd_t (nB_t ancestor unknowns);
// its factor blocks are Dinv_t (nI x nI), L_t (nB x nI) and Lt_t = L_t^T (nI x nB),
// all row-major.  Forward, deepest level first, with Y_I = g_I + F_I:
//   U_t = A_t - L_t Y_I, added into the parent's front
// where F (own rows) and A (boundary rows) collect the children's updates;
// backward, root first:  X_I = Dinv_t Y_I - Lt_t X_B.
// A front entry receives at most two additions onto zero (one per child), so
// the atomic additions give the same sums in any order.  push[u] names where
// update row u goes: the parent's own row -1 - push[u] of F, or row push[u] of A.

__device__ __forceinline__ void nd_push(double2* __restrict__ F, double2* __restrict__ A, int dst, int64_t col,
                                        int R, double2 v) {
  double2* p = dst < 0 ? F + (int64_t)(-1 - dst) * R + col : A + (int64_t)dst * R + col;
  unsafeAtomicAdd(&p->x, v.x);
  unsafeAtomicAdd(&p->y, v.y);
}

// Node tables on the device.
struct NDNodes {
  const int* off;          // [n + 1]
  const int64_t* boff;     // [n + 1] into bnd
  const int* bnd;
  const int64_t* uoff;     // first update row of node t
  const int* push;         // per update row
  const int64_t* mD;       // factor offsets
  const int64_t* mL;
  const int64_t* mLt;
  const double2* fac;
  // several columns: each front row has two slots (one per child) at a fixed
  // column stride ld; update row u of a node goes by a plain store to slot row
  // push2[u] (slot k of the parent's interior row, or of its update row nK + a);
  // slot rows no child writes stay zero from set-up
  const int* push2;
  const int* child;      // [2 n], -1 where absent
  double2* slot;         // [2][nK + urows][ld]
  int64_t ld, srows;     // column stride, rows per slot (nK + urows)
  int nK;
};

// One column: one wave per output row, lanes over the row.
__global__ void __launch_bounds__(NT) k_nd_fwd1(const ND1Fwd* __restrict__ task, int ntask,
                                                const double2* __restrict__ fac, const double2* __restrict__ g,
                                                double2* __restrict__ F, double2* __restrict__ A) {
  const int lane = threadIdx.x & 63;
  // the row is uniform over the wave: its record comes in through scalar loads
  const int q = __builtin_amdgcn_readfirstlane(blockIdx.x * (NT / 64) + (threadIdx.x >> 6));
  if (q >= ntask) return;
  const ND1Fwd tk = task[q];
  const int o = tk.o, nI = tk.nI;
  const double2* Lr = fac + tk.lrow;
  // the accumulated update row is read alongside the operands, not after the sum
  double2 a = make_double2(0.0, 0.0);
  if (lane == 0) a = A[tk.u];
  double ax = 0, ay = 0;
  for (int i = lane; i < nI; i += 64) {
    const double2 m = Lr[i], y0 = g[o + i], y1 = F[o + i];
    const double yx = y0.x + y1.x, yy = y0.y + y1.y;
    ax += m.x * yx - m.y * yy;
    ay += m.x * yy + m.y * yx;
  }
  for (int sh = 32; sh > 0; sh >>= 1) {
    ax += __shfl_xor(ax, sh, 64);
    ay += __shfl_xor(ay, sh, 64);
  }
  if (lane == 0) nd_push(F, A, tk.push, 0, 1, make_double2(a.x - ax, a.y - ay));
}

__global__ void __launch_bounds__(NT) k_nd_bwd1(const ND1Bwd* __restrict__ task, int ntask,
                                                const double2* __restrict__ fac, const int* __restrict__ bnd,
                                                const double2* __restrict__ g, const double2* __restrict__ F,
                                                double2* __restrict__ X) {
  const int lane = threadIdx.x & 63;
  const int q = __builtin_amdgcn_readfirstlane(blockIdx.x * (NT / 64) + (threadIdx.x >> 6));
  if (q >= ntask) return;
  const ND1Bwd tk = task[q];
  const int o = tk.o, nI = tk.nI, nB = tk.nB;
  const double2* Dr = fac + tk.drow;
  const double2* Lr = fac + tk.lrow;
  double ax = 0, ay = 0;
  // the first boundary gather (index, then value) is the longest chain: start it first
  double2 m0 = make_double2(0.0, 0.0), x0 = make_double2(0.0, 0.0);
  if (lane < nB) {
    m0 = Lr[lane];
    x0 = X[bnd[tk.bo + lane]];
  }
  for (int k = lane; k < nI; k += 64) {
    const double2 m = Dr[k], y0 = g[o + k], y1 = F[o + k];
    const double yx = y0.x + y1.x, yy = y0.y + y1.y;
    ax += m.x * yx - m.y * yy;
    ay += m.x * yy + m.y * yx;
  }
  ax -= m0.x * x0.x - m0.y * x0.y;
  ay -= m0.x * x0.y + m0.y * x0.x;
  for (int b = lane + 64; b < nB; b += 64) {
    const double2 m = Lr[b], x = X[bnd[tk.bo + b]];
    ax -= m.x * x.x - m.y * x.y;
    ay -= m.x * x.y + m.y * x.x;
  }
  for (int sh = 32; sh > 0; sh >>= 1) {
    ax += __shfl_xor(ax, sh, 64);
    ay += __shfl_xor(ay, sh, 64);
  }
  if (lane == 0) X[o + tk.i] = make_double2(ax, ay);
}

// Several columns (R <= 64, lane = column): a workgroup owns 32 outputs of a
// node and a range [i0, i1) of the summation (the top levels of the tree hold few
// large nodes, so their sums are split over several workgroups and the partial
// tiles added by k_nd_reduce).  32-row tiles of the factor block go through LDS
// and are read back as wave-wide broadcasts; the operand rows are read coalesced
// (gathered through xidx when given; X2, when given, is added to X).
// acc += sum_i M[i + K j] X_row(i) for this thread's 8 outputs.
__device__ __forceinline__ void nd_mm_core(const double2* __restrict__ M, int K, int i0, int i1, int n_out, int j0,
                                           const double2* __restrict__ X, const double2* __restrict__ X2,
                                           int64_t xbase, const int* __restrict__ xidx, int R, double2 (&acc)[8],
                                           int64_t ld2 = 0, int64_t sst = 0) {
  __shared__ double2 Ms[SMK][SMJ + 1];
  const int r = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool live = r < R;
  for (int ib = i0; ib < i1; ib += SMK) {
    const int nk = min(SMK, i1 - ib);
    for (int e = threadIdx.x; e < SMK * SMJ; e += NT) {
      const int jj = e / SMK, kk = e % SMK;
      Ms[kk][jj] = (kk < nk && j0 + jj < n_out) ? M[(ib + kk) + (int64_t)K * (j0 + jj)] : make_double2(0, 0);
    }
    __syncthreads();
    if (live)
      for (int kk = 0; kk < nk; ++kk) {
        const int64_t row = xidx ? (int64_t)xidx[ib + kk] : xbase + ib + kk;
        double2 x = X[row * R + r];
        if (X2) {
          const double2 x2 = X2[row * ld2 + r], x3 = X2[sst + row * ld2 + r];
          x.x += x2.x + x3.x;
          x.y += x2.y + x3.y;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = cfma(Ms[kk][wv * 8 + t], x, acc[t]);
      }
    __syncthreads();
  }
}

// The same product on the matrix cores for R = 16, 32, 64 columns: each wave
// owns 16 outputs (j tile jt = wave & 1) and two 16-column tiles of R, and
// accumulates complex products as four real FP64 16x16x4 matrix operations per
// step of 4 summation rows (A operand: the 16 operand columns x 4 rows, B
// operand: 4 rows x the 16 outputs of M).  In the result, lane l holds entry
// (row (l >> 4) + 4 v, column l & 15) in its v-th value; the tiles go through
// Dt to the thread-per-column layout of acc used by the callers.

__device__ __forceinline__ void nd_mm_core_mfma(const double2* __restrict__ M, int K, int i0, int i1, int n_out,
                                                int j0, const double2* __restrict__ X,
                                                const double2* __restrict__ X2, int64_t xbase,
                                                const int* __restrict__ xidx, int R, double2 (&acc)[8],
                                                double2* Dt, int64_t ld2 = 0, int64_t sst = 0) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jl = l & 15, kq = l >> 4;
  const int jt = wv & 1, rt0 = (wv >> 1) * 2;
  const int nrt = R >> 4;
  const bool act0 = rt0 < nrt, act1 = rt0 + 1 < nrt;
  const int j = j0 + 16 * jt + jl;
  const bool jv = j < n_out;
  const double2* mcol = M + (int64_t)K * (jv ? j : 0);
  d4 cr0 = {0, 0, 0, 0}, ci0 = {0, 0, 0, 0}, cr1 = {0, 0, 0, 0}, ci1 = {0, 0, 0, 0};
  if (act0) {
    // NU steps of 4 summation rows per pass: every operand load of the pass is
    // issued before its matrix operations (rows past i1 read row i1 - 1, an
    // entry in range, and are zeroed); the operations keep the one-step order
    constexpr int NU = 2;
    for (int k = i0; k < i1; k += 4 * NU) {
      double2 b[NU], a0[NU], a1[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int kk = k + 4 * u + kq;
        const bool kv = kk < i1;
        const int kc = kv ? kk : i1 - 1;
        b[u] = mcol[kc];
        const int64_t row = xidx ? (int64_t)xidx[kc] : xbase + kc;
        const double2* xr = X + row * R + jl;
        a0[u] = xr[16 * rt0];
        a1[u] = act1 ? xr[16 * (rt0 + 1)] : make_double2(0, 0);
        if (X2) {
          // the two child slots of the row
          const double2* x2 = X2 + row * ld2 + jl;
          const double2 c0 = x2[16 * rt0], c1 = x2[sst + 16 * rt0];
          a0[u].x += c0.x + c1.x;
          a0[u].y += c0.y + c1.y;
          if (act1) {
            const double2 d0 = x2[16 * (rt0 + 1)], d1 = x2[sst + 16 * (rt0 + 1)];
            a1[u].x += d0.x + d1.x;
            a1[u].y += d0.y + d1.y;
          }
        }
        if (!(kv && jv)) b[u] = make_double2(0, 0);
        if (!kv) {
          a0[u] = make_double2(0, 0);
          a1[u] = make_double2(0, 0);
        }
      }
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        if (k + 4 * u >= i1) break;   // a step wholly past the range (uniform)
        cr0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u].x, b[u].x, cr0, 0, 0, 0);
        ci0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u].x, b[u].y, ci0, 0, 0, 0);
        cr0 = __builtin_amdgcn_mfma_f64_16x16x4f64(-a0[u].y, b[u].y, cr0, 0, 0, 0);
        ci0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u].y, b[u].x, ci0, 0, 0, 0);
        if (act1) {
          cr1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u].x, b[u].x, cr1, 0, 0, 0);
          ci1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u].x, b[u].y, ci1, 0, 0, 0);
          cr1 = __builtin_amdgcn_mfma_f64_16x16x4f64(-a1[u].y, b[u].y, cr1, 0, 0, 0);
          ci1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u].y, b[u].x, ci1, 0, 0, 0);
        }
      }
    }
    double2* dj = Dt + (16 * jt + jl) * 64;
#pragma unroll
    for (int v = 0; v < 4; ++v) dj[16 * rt0 + kq + 4 * v] = make_double2(cr0[v], ci0[v]);
    if (act1) {
#pragma unroll
      for (int v = 0; v < 4; ++v) dj[16 * (rt0 + 1) + kq + 4 * v] = make_double2(cr1[v], ci1[v]);
    }
  }
  __syncthreads();
  if (l < R) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double2 d = Dt[(wv * 8 + q) * 64 + l];
      acc[q].x += d.x;
      acc[q].y += d.y;
    }
  }
  __syncthreads();
}

// Partial tiles: P[task][32][64].  A task is {node, first output, i0, i1}.
__device__ __forceinline__ void nd_store_part(double2* __restrict__ P, const double2 (&acc)[8], int R) {
  const int r = threadIdx.x & 63, jw = (threadIdx.x >> 6) * 8;
  if (r >= R) return;
  double2* dst = P + (int64_t)blockIdx.x * SMJ * 64;
  for (int q = 0; q < 8; ++q) dst[(jw + q) * 64 + r] = acc[q];
}

// The child slots of front row `row` (interior rows [0, nK), update rows after):
// their sum, or zero at a leaf (no child writes there).
__device__ __forceinline__ double2 nd_slots(const NDNodes& nd, bool leaf, int64_t row, int r) {
  if (leaf) return make_double2(0, 0);
  const double2* p = nd.slot + row * nd.ld + r;
  const double2 a = p[0], b = p[nd.srows * nd.ld];
  return make_double2(a.x + b.x, a.y + b.y);
}

__device__ __forceinline__ bool nd_leaf(const NDNodes& nd, int t) {
  return nd.child[2 * t] < 0 && nd.child[2 * t + 1] < 0;
}

// U_t = A_t - L_t Y_I over the task's range of I (into P when the sum is split);
// Y_I = g_I plus the children's slots, A_t the children's slots of t's update
// rows; U_t goes by plain stores into t's slot of its parent's rows.
template <bool MF>
__global__ void __launch_bounds__(NT) k_nd_fwdR(const int4* __restrict__ task, NDNodes nd,
                                                const double2* __restrict__ g, int R, double2* __restrict__ P) {
  __shared__ double2 Dt[MF ? SMJ * 64 : 1];
  const int4 tk = task[blockIdx.x];
  const int t = tk.x, j0 = tk.y;
  const int o = nd.off[t], nI = nd.off[t + 1] - o;
  const int nB = int(nd.boff[t + 1] - nd.boff[t]);
  const bool leaf = nd_leaf(nd, t);
  const double2* Ys = leaf ? nullptr : nd.slot;
  const int64_t sst = nd.srows * nd.ld;
  double2 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = make_double2(0, 0);
  if (MF) nd_mm_core_mfma(nd.fac + nd.mL[t], nI, tk.z, tk.w, nB, j0, g, Ys, o, nullptr, R, acc, Dt, nd.ld, sst);
  else nd_mm_core(nd.fac + nd.mL[t], nI, tk.z, tk.w, nB, j0, g, Ys, o, nullptr, R, acc, nd.ld, sst);
  if (P) {
    nd_store_part(P, acc, R);
    return;
  }
  const int r = threadIdx.x & 63, jw = j0 + (threadIdx.x >> 6) * 8;
  if (r >= R) return;
  for (int q = 0; q < 8; ++q) {
    const int j = jw + q;
    if (j >= nB) break;
    const int64_t u = nd.uoff[t] + j;
    const double2 a = nd_slots(nd, leaf, nd.nK + u, r);
    nd.slot[(int64_t)nd.push2[u] * nd.ld + r] = make_double2(a.x - acc[q].x, a.y - acc[q].y);
  }
}

// X_I = Dinv_t Y_I - Lt_t X_B; the summation runs over [0, nI) for the first
// product and [nI, nI + nB) for the second, of which the task takes [i0, i1).
template <bool MF>
__global__ void __launch_bounds__(NT) k_nd_bwdR(const int4* __restrict__ task, NDNodes nd,
                                                const double2* __restrict__ g, double2* __restrict__ X, int R,
                                                double2* __restrict__ P) {
  __shared__ double2 Dt[MF ? SMJ * 64 : 1];
  const int4 tk = task[blockIdx.x];
  const int t = tk.x, j0 = tk.y;
  const int o = nd.off[t], nI = nd.off[t + 1] - o;
  const int64_t bo = nd.boff[t];
  const int nB = int(nd.boff[t + 1] - bo);
  const double2* Ys = nd_leaf(nd, t) ? nullptr : nd.slot;
  const int64_t sst = nd.srows * nd.ld;
  double2 a1[8], a2[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a1[q] = a2[q] = make_double2(0, 0);
  const int e1 = min(tk.w, nI);
  const int s2 = max(tk.z, nI) - nI, e2 = tk.w - nI;
  if (MF) {
    if (tk.z < e1) nd_mm_core_mfma(nd.fac + nd.mD[t], nI, tk.z, e1, nI, j0, g, Ys, o, nullptr, R, a1, Dt, nd.ld, sst);
    if (s2 < e2) nd_mm_core_mfma(nd.fac + nd.mLt[t], nB, s2, e2, nI, j0, X, nullptr, 0, nd.bnd + bo, R, a2, Dt);
  } else {
    if (tk.z < e1) nd_mm_core(nd.fac + nd.mD[t], nI, tk.z, e1, nI, j0, g, Ys, o, nullptr, R, a1, nd.ld, sst);
    if (s2 < e2) nd_mm_core(nd.fac + nd.mLt[t], nB, s2, e2, nI, j0, X, nullptr, 0, nd.bnd + bo, R, a2);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) a1[q] = make_double2(a1[q].x - a2[q].x, a1[q].y - a2[q].y);
  if (P) {
    nd_store_part(P, a1, R);
    return;
  }
  const int r = threadIdx.x & 63, jw = j0 + (threadIdx.x >> 6) * 8;
  if (r >= R) return;
  for (int q = 0; q < 8; ++q) {
    const int j = jw + q;
    if (j >= nI) break;
    X[((int64_t)o + j) * R + r] = a1[q];
  }
}

// Sums the S partial tiles of each output tile (tasks q S .. q S + S - 1 share
// node and first output) and finishes the step: U = A - sum stored into the
// parent's slot (forward) or X = sum (backward).
__global__ void k_nd_reduce(const int4* __restrict__ task, int ntiles, int S, const double2* __restrict__ P,
                            NDNodes nd, double2* __restrict__ X, int R, int bwd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ntiles * SMJ * R) return;
  const int r = int(e % R);
  const int jj = int((e / R) % SMJ);
  const int q = int(e / ((int64_t)R * SMJ));
  const int4 tk = task[(int64_t)q * S];
  const int t = tk.x, j = tk.y + jj;
  const int o = nd.off[t], nI = nd.off[t + 1] - o;
  const int n_out = bwd ? nI : int(nd.boff[t + 1] - nd.boff[t]);
  if (j >= n_out) return;
  double sx = 0, sy = 0;
  for (int c = 0; c < S; ++c) {
    const double2 v = P[((int64_t)q * S + c) * SMJ * 64 + jj * 64 + r];
    sx += v.x;
    sy += v.y;
  }
  if (bwd) {
    X[((int64_t)o + j) * R + r] = make_double2(sx, sy);
  } else {
    const int64_t u = nd.uoff[t] + j;
    const double2 a = nd_slots(nd, nd_leaf(nd, t), nd.nK + u, r);
    nd.slot[(int64_t)nd.push2[u] * nd.ld + r] = make_double2(a.x - sx, a.y - sy);
  }
}

// The top depths of the tree as one dense block (several columns): the
// right-hand side of the top unknowns once every deeper node is eliminated,
// r[i] = g[x_i] plus both child slots of each front row listed for x_i
// (its own row in a front of the deepest top depth, and the update rows of
// those fronts that couple to it); x_i = idx[i]; [n][R] and [nK][R] arrays.
__global__ void k_nd_top_gather(int n, const int* __restrict__ idx, const int64_t* __restrict__ gptr,
                                const int* __restrict__ grow, const double2* __restrict__ g,
                                const double2* __restrict__ slot, int64_t ld, int64_t sst, double2* __restrict__ r,
                                int R) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * R) return;
  const int i = int(e / R), c = int(e - (int64_t)i * R);
  double2 v = g[(int64_t)idx[i] * R + c];
  for (int64_t q = gptr[i]; q < gptr[i + 1]; ++q) {
    const double2* p = slot + (int64_t)grow[q] * ld + c;
    const double2 a = p[0], b = p[sst];
    v.x += a.x + b.x;
    v.y += a.y + b.y;
  }
  r[e] = v;
}

// w[x_i] = x[i] for the top unknowns ([n][R] into [nK][R]).
__global__ void k_nd_top_scatter(int n, const int* __restrict__ idx, const double2* __restrict__ x,
                                 double2* __restrict__ w, int R) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * R) return;
  const int i = int(e / R), c = int(e - (int64_t)i * R);
  w[(int64_t)idx[i] * R + c] = x[e];
}

// Set-up of the dense top block: columns k0 .. k0 + cols - 1 of (K^-1) restricted
// to the top unknowns, from the coarse solutions w ([nK][R]) of the unit vectors
// at x_k0 .., into the row-major n x n block M.
__global__ void k_nd_top_collect(int n, const int* __restrict__ idx, const double2* __restrict__ w, int R, int k0,
                                 int cols, double2* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * cols) return;
  const int i = int(e / cols), c = int(e - (int64_t)i * cols);
  M[(int64_t)i * n + k0 + c] = w[(int64_t)idx[i] * R + c];
}

// r = g - K x with K in CSR by row: one wave per row; at one column the lanes
// take the row's entries, otherwise the lanes are the columns.
__global__ void __launch_bounds__(NT) k_csr_residual(int n, const int64_t* __restrict__ ptr,
                                                     const int* __restrict__ col, const double2* __restrict__ val,
                                                     const double2* __restrict__ x, const double2* __restrict__ g,
                                                     double2* __restrict__ r, int R) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t a = ptr[i], b = ptr[i + 1];
  if (R == 1) {
    double ax = 0, ay = 0;
    for (int64_t t = a + lane; t < b; t += 64) {
      const double2 m = val[t], v = x[col[t]];
      ax += m.x * v.x - m.y * v.y;
      ay += m.x * v.y + m.y * v.x;
    }
    for (int sh = 32; sh > 0; sh >>= 1) {
      ax += __shfl_xor(ax, sh, 64);
      ay += __shfl_xor(ay, sh, 64);
    }
    if (lane == 0) r[i] = make_double2(g[i].x - ax, g[i].y - ay);
    return;
  }
  for (int c = lane; c < R; c += 64) {
    double ax = 0, ay = 0;
    for (int64_t t = a; t < b; ++t) {
      const double2 m = val[t], v = x[(int64_t)col[t] * R + c];
      ax += m.x * v.x - m.y * v.y;
      ay += m.x * v.y + m.y * v.x;
    }
    const double2 gg = g[(int64_t)i * R + c];
    r[(int64_t)i * R + c] = make_double2(gg.x - ax, gg.y - ay);
  }
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
// One right-hand side against the symmetric inverse held as its upper 64 x 64
// tiles (I <= J): every tile is read once and serves both the block row I
// (y_I += T x_J) and, transposed, the block row J (y_J += T^T x_I), so the
// coarse step streams half of the dense inverse.  Tile t writes its two
// contributions to fixed places of a partial buffer P[row tile][column tile][64];
// a second kernel adds them per row in a fixed order (no atomics, so repeated
// solves give identical results).

// Packs the upper tiles of K^-1 from the dense row-major inverse, taking
// (A_ij + A_ji) / 2 (the computed inverse is symmetric up to rounding) and
// zero outside n_K.
__global__ void __launch_bounds__(NT) k_pack_sym_tiles(int nK, const double2* __restrict__ A,
                                                       const int2* __restrict__ tij, double2* __restrict__ tiles) {
  const int t = blockIdx.x;
  const int2 IJ = tij[t];
  double2* T = tiles + (int64_t)t * SYM_TILE * SYM_TILE;
  for (int e = threadIdx.x; e < SYM_TILE * SYM_TILE; e += NT) {
    const int i = IJ.x * SYM_TILE + e / SYM_TILE, j = IJ.y * SYM_TILE + e % SYM_TILE;
    double2 v = make_double2(0, 0);
    if (i < nK && j < nK) {
      const double2 a = A[(int64_t)i * nK + j], b = A[(int64_t)j * nK + i];
      v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
    }
    T[e] = v;
  }
}

// SYM_WAVES waves per tile, rows in batches of SYM_KB: lane = column, the
// batch's loads all in flight at once.
constexpr int SYM_KB = 8;

// Exchange steps of the transposed row reduction: with M values per lane the
// partner is the lane across bit 32 M / SYM_KB, and that bit chooses the half
// of the values a lane keeps (and adds the partner's copy to).  The choice is
// made with weights 0 / 1 (exact for finite values) rather than selects, so
// that the values stay in fixed registers.
template <int M>
__device__ __forceinline__ void halve(double* vx, double* vy, int lane) {
  if constexpr (M > 1) {
    constexpr int o = 32 * M / SYM_KB;
    const double fh = (lane & o) ? 1.0 : 0.0, fl = 1.0 - fh;
#pragma unroll
    for (int i = 0; i < M / 2; ++i) {
      const double sx = fh * vx[i] + fl * vx[i + M / 2], sy = fh * vy[i] + fl * vy[i + M / 2];
      const double kx = fl * vx[i] + fh * vx[i + M / 2], ky = fl * vy[i] + fh * vy[i + M / 2];
      vx[i] = kx + __shfl_xor(sx, o, 64);
      vy[i] = ky + __shfl_xor(sy, o, 64);
    }
    halve<M / 2>(vx, vy, lane);
  }
}

// value of lane l (uniform l) in every lane
__device__ __forceinline__ double bcast_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

constexpr int SYM_WAVES = 4;   // waves per tile, each taking SYM_TILE / SYM_WAVES rows

__global__ void __launch_bounds__(SYM_WAVES * 64) k_coarse_symv_tiles(int nK, int nt, const int2* __restrict__ tij,
                                                                      const double2* __restrict__ tiles,
                                                                      const double2* __restrict__ g,
                                                                      double2* __restrict__ P) {
  __shared__ double2 red[SYM_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = blockIdx.x;
  const double2* T = tiles + (int64_t)t * SYM_TILE * SYM_TILE;
  const int2 IJ = tij[t];
  const int jc = IJ.y * SYM_TILE + lane;
  const double2 xJ = jc < nK ? g[jc] : make_double2(0, 0);
  const int ir = IJ.x * SYM_TILE + lane;
  const double2 xIl = ir < nK ? g[ir] : make_double2(0, 0);   // x_I[lane], broadcast per row below
  double cx = 0, cy = 0;
  double2* Prow = P + ((int64_t)IJ.x * nt + IJ.y) * SYM_TILE;
  constexpr int rows = SYM_TILE / SYM_WAVES;
#pragma unroll 1
  for (int r0 = wv * rows; r0 < (wv + 1) * rows; r0 += SYM_KB) {
    double2 a[SYM_KB];
#pragma unroll
    for (int k = 0; k < SYM_KB; ++k) a[k] = T[(r0 + k) * SYM_TILE + lane];
    double vx[SYM_KB], vy[SYM_KB];
#pragma unroll
    for (int k = 0; k < SYM_KB; ++k) {
      vx[k] = a[k].x * xJ.x - a[k].y * xJ.y;
      vy[k] = a[k].x * xJ.y + a[k].y * xJ.x;
      const double xx = bcast_lane(xIl.x, r0 + k), xy = bcast_lane(xIl.y, r0 + k);
      cx += a[k].x * xx - a[k].y * xy;
      cy += a[k].x * xy + a[k].y * xx;
    }
    // row sums over the 64 lanes for the batch's rows at once: recursive halving
    // (each exchange keeps half of the rows, chosen by one bit of the lane), then
    // plain butterfly steps over the low lane bits; lane l ends with row
    // l / (64 / SYM_KB) of the batch
    halve<SYM_KB>(vx, vy, lane);
#pragma unroll
    for (int o = 32 / SYM_KB; o > 0; o >>= 1) {
      vx[0] += __shfl_xor(vx[0], o, 64);
      vy[0] += __shfl_xor(vy[0], o, 64);
    }
    constexpr int low = 64 / SYM_KB;   // lanes sharing one row sum
    if ((lane & (low - 1)) == 0) Prow[r0 + lane / low] = make_double2(vx[0], vy[0]);
  }
  if (IJ.x == IJ.y) return;   // a diagonal tile serves its own block row only
  red[wv][lane] = make_double2(cx, cy);
  __syncthreads();
  if (wv == 0) {
    double sx = 0, sy = 0;
#pragma unroll
    for (int q = 0; q < SYM_WAVES; ++q) {
      sx += red[q][lane].x;
      sy += red[q][lane].y;
    }
    P[((int64_t)IJ.y * nt + IJ.x) * SYM_TILE + lane] = make_double2(sx, sy);
  }
}

// w[I*64 + r] = sum_J P[I][J][r], J in increasing order within each wave's
// share, the four shares added in a fixed order.
__global__ void __launch_bounds__(NT) k_coarse_symv_reduce(int nK, int nt, const double2* __restrict__ P,
                                                           double2* __restrict__ w) {
  __shared__ double2 red[NT / 64][SYM_TILE];
  const int I = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double sx = 0, sy = 0;
  for (int J = wv; J < nt; J += NT / 64) {
    const double2 v = P[((int64_t)I * nt + J) * SYM_TILE + lane];
    sx += v.x;
    sy += v.y;
  }
  red[wv][lane] = make_double2(sx, sy);
  __syncthreads();
  if (wv == 0) {
    double tx = 0, ty = 0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) {
      tx += red[q][lane].x;
      ty += red[q][lane].y;
    }
    const int row = I * SYM_TILE + lane;
    if (row < nK) w[row] = make_double2(tx, ty);
  }
}

// ---------------------------------------------------------------------------
// Full-element separable solve X = Ex [(Ex^T Y Ey) ./ D] Ey^T, one block per (element, RHS).
// One block per (element, chunk of rc right-hand sides): the chunk's n^2 x rc
// entries are staged in shared memory with the right-hand side fastest, so the
// global reads and writes are contiguous runs of rc entries and the four
// products read the shared arrays without bank conflicts.
template <bool SE>
__global__ void __launch_bounds__(NT) k_fdm(const int* __restrict__ elem_cls, const int64_t* __restrict__ dof_off,
                                            const int* __restrict__ cls_n, const int64_t* __restrict__ cls_E,
                                            const int64_t* __restrict__ cls_D, const double2* __restrict__ Ex,
                                            const double2* __restrict__ Ey, const double2* __restrict__ Dinv,
                                            const double2* __restrict__ in, double2* __restrict__ out, int R,
                                            int RCH, const int* __restrict__ cls_nr,
                                            const int* __restrict__ cls_Rm, const int* __restrict__ r_modes,
                                            int zero_coarse, const int* __restrict__ slot_off,
                                            const int64_t* __restrict__ slot_pos, const int* __restrict__ slot_row,
                                            const double* __restrict__ slot_coef, const double2* __restrict__ nu) {
  extern __shared__ double2 sm[];
  const int e = blockIdx.x;
  const int r0 = blockIdx.y * RCH;
  const int rc = min(RCH, R - r0);
  const int c = elem_cls[e];
  const int n = cls_n[c], n2 = n * n, nt = n2 * rc;
  double2* A = sm;
  double2* B = sm + (size_t)n2 * RCH;
  // with SE the class's E_x, E_y and 1/(lambda_x + lambda_y) are staged next to
  // the two stages (the degrees up to 27 let them fit)
  const double2* ex = Ex + cls_E[c];
  const double2* ey = Ey + cls_E[c];
  const double2* di = Dinv + cls_D[c];
  if (SE) {
    double2* exs = B + (size_t)n2 * RCH;
    double2* eys = exs + n2;
    double2* dis = eys + n2;
    for (int idx = threadIdx.x; idx < n2; idx += NT) {
      exs[idx] = ex[idx];
      eys[idx] = ey[idx];
      dis[idx] = di[idx];
    }
    ex = exs;
    ey = eys;
    di = dis;
  }
  const int64_t base = dof_off[e];
  // entry (t, r) of a stage lives at t * rc + r
  for (int idx = threadIdx.x; idx < nt; idx += NT) {
    const int t = idx / rc, r = idx - t * rc;
    A[idx] = in[(base + t) * R + r0 + r];
  }
  __syncthreads();
  if (zero_coarse) {   // uniform over the grid
    const int nr = cls_nr[c];
    const int* rm = r_modes + cls_Rm[c];
    for (int idx = threadIdx.x; idx < nr * rc; idx += NT) {
      const int a = idx / rc, r = idx - a * rc;
      A[rm[a] * rc + r] = make_double2(0, 0);
    }
    if (nu) {   // the element's dual slots (distinct modes, none of them coarse)
      const int s0 = slot_off[e], ns = slot_off[e + 1] - s0;
      for (int idx = threadIdx.x; idx < ns * rc; idx += NT) {
        const int q = idx / rc, r = idx - q * rc, sl = s0 + q;
        const double2 a = nu[(int64_t)slot_row[sl] * R + r0 + r];
        const double cf = slot_coef[sl];
        double2& y = A[(int)(slot_pos[sl] - base) * rc + r];
        y.x -= cf * a.x;
        y.y -= cf * a.y;
      }
    }
    __syncthreads();
  }
  // B = Ex^T A
  for (int idx = threadIdx.x; idx < nt; idx += NT) {
    const int t = idx / rc, r = idx - t * rc, i = t % n, j = t / n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(ex[k + n * i], A[(k + n * j) * rc + r], acc);
    B[idx] = acc;
  }
  __syncthreads();
  // A = (B Ey) .* Dinv
  for (int idx = threadIdx.x; idx < nt; idx += NT) {
    const int t = idx / rc, r = idx - t * rc, i = t % n, j = t / n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(B[(i + n * k) * rc + r], ey[k + n * j], acc);
    A[idx] = cmul(acc, di[t]);
  }
  __syncthreads();
  // B = Ex A
  for (int idx = threadIdx.x; idx < nt; idx += NT) {
    const int t = idx / rc, r = idx - t * rc, i = t % n, j = t / n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(ex[i + n * k], A[(k + n * j) * rc + r], acc);
    B[idx] = acc;
  }
  __syncthreads();
  // out = B Ey^T
  for (int idx = threadIdx.x; idx < nt; idx += NT) {
    const int t = idx / rc, r = idx - t * rc, i = t % n, j = t / n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(B[(i + n * k) * rc + r], ey[j + n * k], acc);
    out[(base + t) * R + r0 + r] = acc;
  }
}

// ---------------------------------------------------------------------------
// The separable element solve on the FP64 matrix cores (n <= 32 modes per
// direction).  One block per (element, RC right-hand sides); the element's
// n^2 x RC coefficients sit in shared memory (entry (a, b, r) of a stage at
// (a + n b) RC + r).  X = Ex [(Ex^T Y Ey) ./ D] Ey^T is four contractions of the
// form D(m, q, r) = sum_k M(m, k) S(k, q, r) over one mode index, each a product
// of a 16 x 4 tile of M (rows m, columns k) with a 4 x 16 tile of the stage
// (rows k, columns (q, r), 16 / RC modes q times RC columns r) on 16x16x4 FP64
// matrix operations: two real operations per step when the class's eigenbasis is
// real (interior elements, the usual case), four when it is complex (impedance
// or layer terms).  Lane l supplies M(m0 + (l & 15), k0 + (l >> 4)) and
// S(k0 + (l >> 4), (q, r) of column l & 15); it receives D(m0 + (l >> 4) + 4 v,
// column l & 15) in value v.  Rows and columns past n are zero operands.
//
// MODE 0: out = A~^-1 in on every element.
// MODE 1: the coarse pass of the element solve of eq. block_matrix_inversion:
//   y = in with the coarse-mode rows zeroed and C_1^T nu subtracted at the dual
//   slots; only the coarse-mode values x_R of A~^-1 y are kept (the algorithmic
//   work is two contractions plus the lines i < 2 and j < 2 of the other two; the
//   kernel runs all four on the matrix cores and reads x_R at the coarse modes,
//   which measured faster than the lines on the vector ALUs) and written to Xr,
//   and GL = K_e x_R (the element's share of -Phi^T y) to GL, both [coarse mode][R].
// MODE 2: the full solve with the Woodbury correction folded in: mu =
//   K_e (x_R - T_e w), and out = A~^-1 (y - E_R mu) (y's coarse rows are zero,
//   so they become -mu), which equals A~^-1 y - G mu.
struct FdmArgs {
  const FdmRec* rec;
  const int* order;   // elements grouped by class
  const int* elem_cls;
  const int64_t* dof_off;
  const int* cls_n;
  const int64_t* cls_E;
  const int64_t* cls_D;
  const double2* Ex;
  const double2* Ey;
  const double2* Dinv;
  const int* cls_real;   // per class: 1 when Ex and Ey are real
  const double2* in;
  double2* out;
  int R;
  const int* cls_nr;
  const int* cls_R;
  const int* r_modes;
  int zero_coarse;
  const int* slot_off;
  const int64_t* slot_pos;
  const int* slot_row;
  const double* slot_coef;
  const double2* nu;
  const int* cm_off;
  const int64_t* cls_Kc;
  const double2* Kc;
  double2* Xr;
  double2* GL;
  const int* t_ptr;
  const int* t_dof;
  const double* t_coef;
  const double2* w;
  // mode 2: K_e x_R given ([ncm][R]; Xr then holds -T_e w), the correction
  // formed as K_e x_R - K_e T_e w
  const double2* kx;
  // mode 1: the dual-slot values of A~^-1 y as well ([nslots][R])
  double2* xslot;
};

// D = M S over one mode index (see above), for classes of n <= NP modes (NP 16
// or 32).  KF_IN: the contraction index is the fast index of S's positions;
// KF_OUT: m is the fast index of D's positions; MFAST: M(m, k) = mat[m + LD k],
// else mat[m LD + k] with LD = NP + 1 (the eigenbases are staged zero-padded to
// NP x NP in columns of NP + 1 entries, which keeps the operand reads free of
// shared-memory bank conflicts; rows
// and columns past n multiply by zero; every stage position up to NP^2 holds a
// finite value, so no operand needs a bounds test).  With scale, D is
// multiplied entrywise by scale at position (q + n m) (1 / (lambda_x + lambda_y)
// in the second contraction, whose output keeps i = q fast).
template <int RC, int NP, bool CPLX, bool KF_IN, bool KF_OUT, bool MFAST>
__device__ __forceinline__ void fdm_contract(const double2* __restrict__ mat, const double2* __restrict__ S,
                                             double2* __restrict__ D, int n, const double2* __restrict__ scale) {
  constexpr int QT = 16 / RC;                   // modes q per column tile
  constexpr int MT = NP / 16;                   // row tiles
  constexpr int KS = NP / 4;                    // steps of four summation indices
  constexpr int TMAX = MT * (NP / QT);          // tiles when n = NP
  constexpr int TPW = (TMAX + 3) / 4;           // tiles per wave (every wave runs all of its
                                                // slots in straight-line code; a slot past the
                                                // last tile repeats it and is not stored)
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c16 = l & 15, kq = l >> 4;
  const int qo = c16 / RC, r = c16 % RC;
  const int ntiles = (n + QT - 1) / QT, T = MT * ntiles;
  constexpr int LD = NP + 1;                    // eigenbasis leading dimension (odd: no bank conflicts)
  const int sstep = KF_IN ? 4 * RC : 4 * n * RC;   // operand step per four summation indices
  d4 cr[TPW], ci[TPW];
  const double2* ap[TPW];
  const double2* bp[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    cr[u] = (d4){0, 0, 0, 0};
    ci[u] = (d4){0, 0, 0, 0};
    const int tile = min(wv + 4 * u, T - 1);
    const int nt = tile / MT, mt = tile - nt * MT;
    const int m = 16 * mt + c16, q = nt * QT + qo;
    ap[u] = mat + (MFAST ? m + LD * kq : m * LD + kq);
    bp[u] = S + (KF_IN ? kq + n * q : q + n * kq) * RC + r;
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const double2 a = ap[u][MFAST ? 4 * ks * LD : 4 * ks];
      const double2 b = bp[u][ks * sstep];
      cr[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr[u], 0, 0, 0);
      ci[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci[u], 0, 0, 0);
      if (CPLX) {
        cr[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr[u], 0, 0, 0);
        ci[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci[u], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int tile = wv + 4 * u;
    const int nt = tile / MT, mt = tile - nt * MT;
    const int q = nt * QT + qo;
    if (tile < T && q < n) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * mt + kq + 4 * v;
        if (m < n) {
          const int pos = KF_OUT ? m + n * q : q + n * m;
          double2 o = make_double2(cr[u][v], ci[u][v]);
          if (scale) o = cmul(o, scale[pos]);
          D[pos * RC + r] = o;
        }
      }
    }
  }
}

// W = (Ex^T Y Ey) ./ D from A into A (B as the intermediate stage).
template <int RC, int NP, bool CPLX>
__device__ __forceinline__ void fdm_forward(const double2* ex, const double2* ey, const double2* di, double2* A,
                                            double2* B, int n) {
  // B(i, iy) = sum_ix Ex(ix, i) Y(ix, iy): M(m = i, k = ix) = Ex(ix, i) at ix + LD i
  fdm_contract<RC, NP, CPLX, true, true, false>(ex, A, B, n, nullptr);
  __syncthreads();
  // W(i, j) = sum_iy B(i, iy) Ey(iy, j): M(m = j, k = iy) = Ey(iy, j) at iy + LD j
  fdm_contract<RC, NP, CPLX, false, false, false>(ey, B, A, n, di);
  __syncthreads();
}

// X = Ex W Ey^T from A into A.
template <int RC, int NP, bool CPLX>
__device__ __forceinline__ void fdm_backward(const double2* ex, const double2* ey, double2* A, double2* B, int n) {
  // Z(i', j) = sum_i Ex(i', i) W(i, j): M(m = i', k = i) at i' + LD i
  fdm_contract<RC, NP, CPLX, true, true, true>(ex, A, B, n, nullptr);
  __syncthreads();
  // X(i', j') = sum_j Z(i', j) Ey(j', j): M(m = j', k = j) at j' + LD j
  fdm_contract<RC, NP, CPLX, false, false, true>(ey, B, A, n, nullptr);
  __syncthreads();
}

template <int RC, int NP>
__device__ __forceinline__ void fdm_forward_any(bool real_e, const double2* ex, const double2* ey,
                                                const double2* di, double2* A, double2* B, int n) {
  if (real_e) fdm_forward<RC, NP, false>(ex, ey, di, A, B, n);
  else fdm_forward<RC, NP, true>(ex, ey, di, A, B, n);
}

template <int RC, int NP>
__device__ __forceinline__ void fdm_backward_any(bool real_e, const double2* ex, const double2* ey, double2* A,
                                                 double2* B, int n) {
  if (real_e) fdm_backward<RC, NP, false>(ex, ey, A, B, n);
  else fdm_backward<RC, NP, true>(ex, ey, A, B, n);
}

// Shared memory of k_fdm_mf (double2 entries): two stages, the padded Ex and Ey
// (NPMAX (NPMAX + 1) each), 1 / D (nmax^2), x_R (nrmax RC) and, for the two
// passes of the element solve, K_e (nrmax^2).
// Stage entries per column: the operand reads of a contraction reach position
// n NP + NP + 16 at most (summation indices up to NP - 1, modes q up to the last
// column tile), so a stage of that many positions per column, zero past n^2,
// needs no bounds tests.
__host__ __device__ inline int fdm_stage(int nmax, int npmax) { return nmax * npmax + npmax + 16; }

__host__ __device__ inline size_t fdm_mf_entries(int nmax, int npmax, int nrmax, int rc, bool coarse) {
  return size_t(2) * fdm_stage(nmax, npmax) * rc + size_t(2) * npmax * (npmax + 1) + size_t(nmax) * nmax +
         size_t(nrmax) * rc + (coarse ? size_t(nrmax) * nrmax : 0);
}

// Loads of one item's coefficients kept in registers: entry i = threadIdx.x +
// u NT of the item's n^2 x RC stage (the batch covers n^2 RC <= fdm_fb(RC) NT;
// larger stages load the rest when they are staged).  At 16 columns a block
// holds the compute unit's shared memory alone (one wave per SIMD), so the
// batch takes 12 entries and covers a 13x13 element; narrower items run two
// blocks per compute unit and keep 8 (the register file of two waves per SIMD).
constexpr int FDM_FB = 8;   // batch of the staging loops
__host__ __device__ constexpr int fdm_fb(int rc) { return rc >= 16 ? 12 : FDM_FB; }

template <int RC>
__device__ __forceinline__ void fdm_prefetch(const FdmArgs& g, int e, int r0, double2 (&v)[fdm_fb(RC)]) {
  const FdmRec fr = g.rec[e];
  const int ny = fr.n * fr.n * RC, R = g.R, rc = min(RC, R - r0);
  const double2* __restrict__ in = g.in + fr.base * R + r0;
#pragma unroll
  for (int u = 0; u < fdm_fb(RC); ++u) {
    const int i = threadIdx.x + u * NT;
    const int t = i / RC, r = i - t * RC;
    v[u] = (i < ny && r < rc) ? in[(int64_t)t * R + r] : make_double2(0, 0);
  }
}

// One (element, RC columns) item of k_fdm_mf.  v holds the item's prefetched
// coefficients and receives the next item's (next_e >= 0) once they are staged;
// load_e: stage the class's eigenbases (skipped when the block's previous item
// had the same class).
template <int RC, int MODE, int NPMAX>
__device__ __forceinline__ void fdm_item(const FdmArgs& g, int nmax, int nrmax, double2* sm, int e, int r0,
                                         bool load_e, double2 (&v)[fdm_fb(RC)], int next_e, int next_r0) {
  const int R = g.R;
  const int rc = min(RC, R - r0);
  const FdmRec fr = g.rec[e];   // one record per element: offsets and sizes of its class
  const int n = fr.n, n2 = n * n;
  const int np = (NPMAX == 32 && n > 16) ? 32 : 16;   // padding of this element's class
  const int ld = np + 1;
  const int nst = fdm_stage(nmax, NPMAX) * RC;
  double2* A = sm;
  double2* B = sm + nst;
  double2* exs = B + nst;
  double2* eys = exs + NPMAX * (NPMAX + 1);
  double2* dis = eys + NPMAX * (NPMAX + 1);
  double2* xs = dis + nmax * nmax;     // nrmax x RC: x_R (pass 1) or x_R - T w (pass 2)
  double2* ks = xs + nrmax * RC;       // nrmax x nrmax: K_e (passes 1 and 2)
  const bool real_e = fr.real != 0;
  const int64_t base = fr.base;
  const int nr = fr.nr;
  const int cmo = fr.cmo;
  // pass 2: x_R - T_e w of the thread's coarse-mode entries (formed by
  // k_coarse_minus_tw), loaded before the staging
  double2 gx[2] = {make_double2(0, 0), make_double2(0, 0)};
  double2 gk[2] = {make_double2(0, 0), make_double2(0, 0)};   // K_e x_R when given
  if (MODE == 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = threadIdx.x + u * NT, a = idx / RC, r = idx - a * RC;
      if (a < nr && r < rc) {
        gx[u] = g.Xr[(int64_t)(cmo + a) * R + r0 + r];
        if (g.kx) gk[u] = g.kx[(int64_t)(cmo + a) * R + r0 + r];
      }
    }
  }
  const int ny = n2 * RC;
  // the prefetched coefficients, then (only for stages larger than the
  // prefetch) the rest, loads batched; the stage tails past n^2 are zero
#pragma unroll
  for (int u = 0; u < fdm_fb(RC); ++u) {
    const int i = threadIdx.x + u * NT;
    if (i < ny) A[i] = v[u];
  }
  {
    const double2* __restrict__ in = g.in + base * R + r0;
    for (int i0 = threadIdx.x + fdm_fb(RC) * NT; i0 < ny; i0 += NT * FDM_FB) {
      double2 w[FDM_FB];
#pragma unroll
      for (int u = 0; u < FDM_FB; ++u) {
        const int i = i0 + u * NT;
        const int t = i / RC, r = i - t * RC;
        w[u] = (i < ny && r < rc) ? in[(int64_t)t * R + r] : make_double2(0, 0);
      }
#pragma unroll
      for (int u = 0; u < FDM_FB; ++u) {
        const int i = i0 + u * NT;
        if (i < ny) A[i] = w[u];
      }
    }
  }
  if (load_e) {
    // eigenbases zero-padded to np x np in columns of ld entries, 1 / D and,
    // for the two passes, K_e
    const double2* __restrict__ ex = g.Ex + fr.eoff;
    const double2* __restrict__ ey = g.Ey + fr.eoff;
    const double2* __restrict__ di = g.Dinv + fr.doff;
    const double2* __restrict__ kc = g.Kc + fr.kc;
    const int ne = np * ld, count = 2 * ne + n2 + (MODE != 0 ? nr * nr : 0);
    for (int i0 = threadIdx.x; i0 < count; i0 += NT * FDM_FB) {
      double2 w[FDM_FB];
#pragma unroll
      for (int u = 0; u < FDM_FB; ++u) {
        const int j = i0 + u * NT;
        w[u] = make_double2(0, 0);
        if (j < 2 * ne) {
          const int w2 = j >= ne, jj = j - w2 * ne;
          const int a = jj % ld, b = jj / ld;
          if (a < n && b < n) w[u] = (w2 ? ey : ex)[a + n * b];
        } else if (j < 2 * ne + n2) {
          w[u] = di[j - 2 * ne];
        } else if (j < count) {
          w[u] = kc[j - 2 * ne - n2];
        }
      }
#pragma unroll
      for (int u = 0; u < FDM_FB; ++u) {
        const int j = i0 + u * NT;
        if (j < ne) exs[j] = w[u];
        else if (j < 2 * ne) eys[j - ne] = w[u];
        else if (j < 2 * ne + n2) dis[j - 2 * ne] = w[u];
        else if (j < count) ks[j - 2 * ne - n2] = w[u];
      }
    }
  }
  for (int i = ny + threadIdx.x; i < fdm_stage(n, np) * RC; i += NT) {
    A[i] = make_double2(0, 0);
    B[i] = make_double2(0, 0);
  }
  // the next item's coefficients are loaded while this one computes
  if (next_e >= 0) fdm_prefetch<RC>(g, next_e, next_r0, v);
  const int* rm = g.r_modes + fr.roff;
  if (MODE == 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = threadIdx.x + u * NT;
      if (idx < nr * RC) xs[idx] = gx[u];
    }
    for (int idx = threadIdx.x + 2 * NT; idx < nr * RC; idx += NT) {
      const int a = idx / RC, r = idx - a * RC;
      xs[idx] = r < rc ? g.Xr[(int64_t)(cmo + a) * R + r0 + r] : make_double2(0, 0);
    }
  }
  __syncthreads();
  if (g.zero_coarse) {   // uniform over the grid
    for (int idx = threadIdx.x; idx < nr * RC; idx += NT) {
      const int a = idx / RC, r = idx - a * RC;
      double2 y = make_double2(0, 0);
      if (MODE == 2) {   // -mu = -K_e (x_R - T_e w), or K_e T_e w - K_e x_R from kx
        for (int b = 0; b < nr; ++b) y = cfma(ks[a + nr * b], xs[b * RC + r], y);
        y.x = -y.x;
        y.y = -y.y;
        if (g.kx) {
          const int u = (idx - (int)threadIdx.x) / NT;
          double2 k = make_double2(0, 0);
          if (u == 0) k = gk[0];
          else if (u == 1) k = gk[1];
          else if (r < rc) k = g.kx[(int64_t)(cmo + a) * R + r0 + r];
          y.x -= k.x;
          y.y -= k.y;
        }
      }
      A[rm[a] * RC + r] = y;
    }
    if (g.nu) {   // the element's dual slots (distinct modes, none of them coarse)
      const int s0 = fr.s0, ns = fr.s1 - s0;
      for (int idx = threadIdx.x; idx < ns * rc; idx += NT) {
        const int q = idx / rc, r = idx - q * rc, sl = s0 + q;
        const double2 a = g.nu[(int64_t)g.slot_row[sl] * R + r0 + r];
        const double cf = g.slot_coef[sl];
        double2& y = A[(int)(g.slot_pos[sl] - base) * RC + r];
        y.x -= cf * a.x;
        y.y -= cf * a.y;
      }
    }
    __syncthreads();
  }
  if (NPMAX == 32 && np == 32) fdm_forward_any<RC, NPMAX>(real_e, exs, eys, dis, A, B, n);
  else fdm_forward_any<RC, 16>(real_e, exs, eys, dis, A, B, n);
  if (NPMAX == 32 && np == 32) fdm_backward_any<RC, NPMAX>(real_e, exs, eys, A, B, n);
  else fdm_backward_any<RC, 16>(real_e, exs, eys, A, B, n);
  if (MODE == 1) {
    // x_R (the coarse-mode values of A~^-1 y) and GL = K_e x_R
    for (int idx = threadIdx.x; idx < nr * RC; idx += NT) {
      const int a = idx / RC, r = idx - a * RC;
      const double2 x = A[rm[a] * RC + r];
      xs[idx] = x;
      if (r < rc) g.Xr[(int64_t)(cmo + a) * R + r0 + r] = x;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nr * rc; idx += NT) {
      const int a = idx / rc, r = idx - a * rc;
      double2 acc = make_double2(0, 0);
      for (int b = 0; b < nr; ++b) acc = cfma(ks[a + nr * b], xs[b * RC + r], acc);
      g.GL[(int64_t)(cmo + a) * R + r0 + r] = acc;
    }
    if (g.xslot) {   // the element's dual slots (distinct modes, none of them coarse)
      const int s0 = fr.s0, ns = fr.s1 - s0;
      for (int idx = threadIdx.x; idx < ns * rc; idx += NT) {
        const int q = idx / rc, r = idx - q * rc, sl = s0 + q;
        g.xslot[(int64_t)sl * R + r0 + r] = A[(int)(g.slot_pos[sl] - base) * RC + r];
      }
    }
    return;
  }
  double2* __restrict__ out = g.out + base * R + r0;
  for (int idx = threadIdx.x; idx < n2 * rc; idx += NT) {
    const int t = idx / rc, r = idx - t * rc;
    out[(int64_t)t * R + r] = A[t * RC + r];
  }
}

// The element solves as a persistent grid: each block takes the items (element
// in class order, chunk of RC columns) blockIdx.x, blockIdx.x + gridDim.x, ...
// (short-lived blocks would leave most compute units waiting on workgroup
// dispatch); a block re-stages the eigenbases only when the class changes.
template <int RC, int MODE, int NPMAX>
__global__ void __launch_bounds__(NT) k_fdm_mf(FdmArgs g, int nmax, int nrmax, int nitems, int nchunk) {
  extern __shared__ double2 sm[];
  int cur = -1;
  double2 v[fdm_fb(RC)];
  int it = blockIdx.x;
  int e = -1, r0 = 0;
  if (it < nitems) {
    const int pos = it / nchunk;
    e = g.order[pos];
    r0 = (it - pos * nchunk) * RC;
    fdm_prefetch<RC>(g, e, r0, v);
  }
  for (; it < nitems; it += gridDim.x) {
    const int itn = it + gridDim.x;
    int ne = -1, nr0 = 0;
    if (itn < nitems) {
      const int pos = itn / nchunk;
      ne = g.order[pos];
      nr0 = (itn - pos * nchunk) * RC;
    }
    const int c = g.rec[e].cls;
    fdm_item<RC, MODE, NPMAX>(g, nmax, nrmax, sm, e, r0, c != cur, v, ne, nr0);
    cur = c;
    e = ne;
    r0 = nr0;
    __syncthreads();   // the next item overwrites the stages
  }
}

// Xr[i][r] -= sum_t T(i, t) w[t][r] for every coarse mode i (its expansion over
// the coarse unknowns): the x_R - T_e w of the corrected element solve (-T_e w
// with from_zero).
__global__ void __launch_bounds__(NT) k_coarse_minus_tw(int ncm, int R, const int* __restrict__ t_ptr,
                                                        const int* __restrict__ t_dof,
                                                        const double* __restrict__ t_coef,
                                                        const double2* __restrict__ w, double2* __restrict__ Xr,
                                                        int from_zero) {
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx >= (int64_t)ncm * R) return;
  const int i = int(idx / R), r = int(idx - (int64_t)i * R);
  double2 x = from_zero ? make_double2(0, 0) : Xr[idx];
  for (int t = t_ptr[i]; t < t_ptr[i + 1]; ++t) {
    const double2 ww = w[(int64_t)t_dof[t] * R + r];
    x.x -= t_coef[t] * ww.x;
    x.y -= t_coef[t] * ww.y;
  }
  Xr[idx] = x;
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

// mu = Kc (c - T_e w); X -= G mu.  Afterwards X at the coarse modes equals T_e w
// (T_e w: each coarse mode's expansion over the global coarse unknowns).
// Woodbury correction of the full-element solves, one block per (element, chunk
// of rc right-hand sides), right-hand side fastest as in k_fdm: the removed
// modes' values minus their coarse parts, times K_e, then X -= G mu.
__global__ void __launch_bounds__(NT) k_correct(const int* __restrict__ elem_cls, const int64_t* __restrict__ dof_off,
                                                const int* __restrict__ cm_off, const int* __restrict__ cls_n,
                                                const int* __restrict__ cls_nr, const int* __restrict__ cls_R,
                                                const int* __restrict__ r_modes, const int64_t* __restrict__ cls_Kc,
                                                const double2* __restrict__ Kc, const int64_t* __restrict__ cls_G,
                                                const double2* __restrict__ G, const int* __restrict__ t_ptr,
                                                const int* __restrict__ t_dof, const double* __restrict__ t_coef,
                                                double2* __restrict__ X, const double2* __restrict__ w, int R,
                                                int RCH) {
  extern __shared__ double2 sm[];
  const int e = blockIdx.x;
  const int r0 = blockIdx.y * RCH;
  const int rc = min(RCH, R - r0);
  const int c = elem_cls[e];
  const int n = cls_n[c], n2 = n * n, nr = cls_nr[c];
  double2* dv = sm;                          // nr x rc
  double2* mu = sm + (size_t)NRMAX * RCH;    // nr x rc
  const int* rm = r_modes + cls_R[c];
  const int64_t base = dof_off[e];
  for (int idx = threadIdx.x; idx < nr * rc; idx += NT) {
    const int a = idx / rc, r = idx - a * rc;
    double2 x = X[(base + rm[a]) * R + r0 + r];
    const int i = cm_off[e] + a;
    for (int t = t_ptr[i]; t < t_ptr[i + 1]; ++t) {
      const double2 ww = w[(int64_t)t_dof[t] * R + r0 + r];
      x.x -= t_coef[t] * ww.x;
      x.y -= t_coef[t] * ww.y;
    }
    dv[idx] = x;
  }
  __syncthreads();
  const double2* K = Kc + cls_Kc[c];
  for (int idx = threadIdx.x; idx < nr * rc; idx += NT) {
    const int a = idx / rc, r = idx - a * rc;
    double2 acc = make_double2(0, 0);
    for (int b = 0; b < nr; ++b) acc = cfma(K[a + nr * b], dv[b * rc + r], acc);
    mu[idx] = acc;
  }
  __syncthreads();
  const double2* Gc = G + cls_G[c];
  for (int idx = threadIdx.x; idx < n2 * rc; idx += NT) {
    const int t = idx / rc, r = idx - t * rc;
    double2 acc = X[(base + t) * R + r0 + r];
    for (int a = 0; a < nr; ++a) {
      const double2 gm = cmul(Gc[t + (int64_t)n2 * a], mu[a * rc + r]);
      acc.x -= gm.x;
      acc.y -= gm.y;
    }
    X[(base + t) * R + r0 + r] = acc;
  }
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

// Far field, step 1: trace u and normal derivative d_n' u at the Gauss nodes of
// every boundary side of the enclosed region (Sec. 3.3.1), one block per
// (side, RHS).  For a side normal to x the trace row of the vertex-basis
// coefficients is X[a0, b] (a0 = 0 at x = +1, 1 at x = -1) and the normal
// derivative uses dN~_a(+-1); sides normal to y swap the roles.
__global__ void __launch_bounds__(NT) k_far_trace(const int* __restrict__ elem, const int* __restrict__ side,
                                                  const int* __restrict__ node_off, const int64_t* __restrict__ tab_off,
                                                  const double* __restrict__ tab, const double* __restrict__ dscale,
                                                  const int* __restrict__ elem_cls, const int* __restrict__ cls_n,
                                                  const int64_t* __restrict__ dof_off, const double2* __restrict__ X,
                                                  int R, double2* __restrict__ U, double2* __restrict__ DU) {
  __shared__ double2 tv[64], dv[64];
  const int g = blockIdx.x, r = blockIdx.y;
  const int e = elem[g], sd = side[g];
  const int n = cls_n[elem_cls[e]];
  const int64_t base = dof_off[e];
  // tab for this side: [q][n] basis values at the nodes, then dN~(end) (n values)
  const int q0 = node_off[g], nq = node_off[g + 1] - q0;
  const double* Nq = tab + tab_off[g];
  const double* dend = Nq + (int64_t)nq * n;
  const bool xside = sd <= 2;
  const int a0 = (sd == 2 || sd == 4) ? 0 : 1;
  for (int b = threadIdx.x; b < n; b += NT) {
    double2 t = xside ? X[(base + a0 + (int64_t)n * b) * R + r] : X[(base + b + (int64_t)n * a0) * R + r];
    double dx = 0, dy = 0;
    for (int a = 0; a < n; ++a) {
      double2 c = xside ? X[(base + a + (int64_t)n * b) * R + r] : X[(base + b + (int64_t)n * a) * R + r];
      dx += dend[a] * c.x;
      dy += dend[a] * c.y;
    }
    tv[b] = t;
    dv[b] = make_double2(dx * dscale[g], dy * dscale[g]);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nq; q += NT) {
    double ux = 0, uy = 0, vx = 0, vy = 0;
    for (int b = 0; b < n; ++b) {
      double w = Nq[(int64_t)q * n + b];
      ux += w * tv[b].x;
      uy += w * tv[b].y;
      vx += w * dv[b].x;
      vy += w * dv[b].y;
    }
    U[(int64_t)(q0 + q) * R + r] = make_double2(ux, uy);
    DU[(int64_t)(q0 + q) * R + r] = make_double2(vx, vy);
  }
}

// Far field, step 2: E[r][phi] = sum_q w_q e^{-i k xhat.x_q} [(xhat.n'_q) U_q + (i k)^-1 DU_q].
__global__ void __launch_bounds__(NT) k_far_sum(int nq, const double* __restrict__ px, const double* __restrict__ py,
                                                const double* __restrict__ pw, const double* __restrict__ pnx,
                                                const double* __restrict__ pny, const double* __restrict__ ang,
                                                double k, const double2* __restrict__ U, const double2* __restrict__ DU,
                                                int R, int nrhs_out, int nfar, double2* __restrict__ E) {
  __shared__ double2 red[NT];
  const int f = blockIdx.x;
  const double cx = cos(ang[f]), cy = sin(ang[f]);
  const int r = threadIdx.x % R, rl = threadIdx.x / R, step = NT / R;
  double ax = 0, ay = 0;
  for (int q = rl; q < nq; q += step) {
    double ph = -k * (cx * px[q] + cy * py[q]);
    double c = cos(ph), s = sin(ph);
    double xn = cx * pnx[q] + cy * pny[q];
    double2 u = U[(int64_t)q * R + r], du = DU[(int64_t)q * R + r];
    // (i k)^-1 du = -i du / k
    double tx = xn * u.x + du.y / k, ty = xn * u.y - du.x / k;
    ax += pw[q] * (c * tx - s * ty);
    ay += pw[q] * (c * ty + s * tx);
  }
  double2 t = block_sum_by_rhs(make_double2(ax, ay), R, red);
  if (threadIdx.x < R && threadIdx.x < nrhs_out) E[(int64_t)threadIdx.x * nfar + f] = t;
}

// Plane-wave loads in the vertex basis, one block per (listed element, RHS):
// scattered field, f = k^2 (eps - 1) e^{ik d.x} (separable: b = f0 a (x) b);
// total field, impedance data g = ik(d.n - 1) e^{ik d.x} on the boundary sides.
// Nq holds the vertex basis at the element degree's Gauss nodes ([q][n]).
__global__ void __launch_bounds__(NT) k_plane_wave_loads(
    int kind, const int* __restrict__ elems, const int* __restrict__ elem_cls, const int* __restrict__ cls_n,
    const int64_t* __restrict__ dof_off, const int* __restrict__ cls_q, const int64_t* __restrict__ cls_qoff,
    const double* __restrict__ qx, const double* __restrict__ qw, const double* __restrict__ qN,
    const double* __restrict__ ox, const double* __restrict__ oy, const double* __restrict__ hx,
    const double* __restrict__ hy, const double* __restrict__ eps, const int* __restrict__ bmask,
    const double* __restrict__ angles, double k, double2* __restrict__ B, int R) {
  __shared__ double2 a[64], b[64], sv[4][64];
  const int e = elems[blockIdx.x], r = blockIdx.y;
  const int c = elem_cls[e], n = cls_n[c], q = cls_q[c];
  const double* xq = qx + cls_qoff[c];
  const double* wq = qw + cls_qoff[c];
  const double* N = qN + cls_qoff[c] * 64;   // [q][64], basis padded to 64 columns
  const double dx = cos(angles[r]), dy = sin(angles[r]);
  const double X0 = ox[e], Y0 = oy[e], HX = hx[e], HY = hy[e];
  const int64_t base = dof_off[e];
  if (kind == 2) {
    for (int m = threadIdx.x; m < 2 * n; m += NT) {
      const bool yd = m >= n;
      const int mm = yd ? m - n : m;
      double sx = 0, sy = 0;
      for (int t = 0; t < q; ++t) {
        double pos = yd ? Y0 + (xq[t] + 1) * HY / 2 : X0 + (xq[t] + 1) * HX / 2;
        double ph = k * (yd ? dy : dx) * pos;
        double wn = wq[t] * N[(int64_t)t * 64 + mm];
        sx += wn * cos(ph);
        sy += wn * sin(ph);
      }
      if (yd) b[mm] = make_double2(sx, sy); else a[mm] = make_double2(sx, sy);
    }
    __syncthreads();
    const double f0 = k * k * (eps[e] - 1.0) * (HX / 2) * (HY / 2);
    for (int t = threadIdx.x; t < n * n; t += NT) {
      int ix = t % n, iy = t / n;
      double2 p = cmul(a[ix], b[iy]);
      B[(base + t) * R + r] = make_double2(f0 * p.x, f0 * p.y);
    }
  } else {
    for (int t = threadIdx.x; t < n * n; t += NT) B[(base + t) * R + r] = make_double2(0, 0);
    for (int m = threadIdx.x; m < 4 * n; m += NT) {
      const int sd = m / n + 1, mm = m % n;
      double sx = 0, sy = 0;
      if (bmask[e] & (1 << (sd - 1))) {
        const double nx = sd == 1 ? -1 : sd == 2 ? 1 : 0, ny = sd == 3 ? -1 : sd == 4 ? 1 : 0;
        const double hl = sd <= 2 ? HY : HX;
        const double gx = 0, gy = k * (dx * nx + dy * ny - 1.0);   // ik(d.n - 1)
        for (int t = 0; t < q; ++t) {
          double x, y;
          if (sd <= 2) { x = sd == 1 ? X0 : X0 + HX; y = Y0 + (xq[t] + 1) * HY / 2; }
          else { y = sd == 3 ? Y0 : Y0 + HY; x = X0 + (xq[t] + 1) * HX / 2; }
          double ph = k * (dx * x + dy * y);
          double cr = cos(ph), ci = sin(ph);
          double wn = wq[t] * (hl / 2) * N[(int64_t)t * 64 + mm];
          sx += wn * (gx * cr - gy * ci);
          sy += wn * (gx * ci + gy * cr);
        }
      }
      sv[sd - 1][mm] = make_double2(sx, sy);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      // scatter the four side vectors onto the trace modes (left: ix=1, right: ix=0,
      // bottom: iy=1, top: iy=0); corners receive two contributions
      for (int sd = 1; sd <= 4; ++sd) {
        if (!(bmask[e] & (1 << (sd - 1)))) continue;
        for (int mm = 0; mm < n; ++mm) {
          int64_t pos = sd == 1 ? 1 + (int64_t)n * mm : sd == 2 ? (int64_t)n * mm : sd == 3 ? mm + n : mm;
          double2& dst = B[(base + pos) * R + r];
          dst.x += sv[sd - 1][mm].x;
          dst.y += sv[sd - 1][mm].y;
        }
      }
    }
  }
}

// Adjoint gradient with respect to each element's relative permittivity:
//   dJ/d eps_e = 2 Re( conj(E) [ lambda_e^T db_e + k^2 (h_x h_y / 4) lambda_e^T (M~ (x) M~) u_e ] )
// with db_e = k^2 (h_x/2)(h_y/2) a (x) b the scattered-field load per unit (eps_e - 1)
// (a, b: the 1-D integrals of N~ e^{ik d x} as in the plane-wave loads).  One block per element.
__global__ void __launch_bounds__(NT) k_eps_grad(
    const int* __restrict__ elem_cls, const int* __restrict__ cls_n, const int64_t* __restrict__ dof_off,
    const int* __restrict__ cls_q, const int64_t* __restrict__ cls_qoff, const double* __restrict__ qx,
    const double* __restrict__ qw, const double* __restrict__ qN, const double* __restrict__ cls_M,
    const int64_t* __restrict__ cls_Moff, const double* __restrict__ ox, const double* __restrict__ oy,
    const double* __restrict__ hx, const double* __restrict__ hy, const double2* __restrict__ mass_fac,
    const double2* __restrict__ U, const double2* __restrict__ Lam, double2 E, double k, double dx, double dy,
    double* __restrict__ grad) {
  extern __shared__ double2 sm[];
  __shared__ double2 red[NT];
  const int e = blockIdx.x;
  const int c = elem_cls[e], n = cls_n[c], n2 = n * n, q = cls_q[c];
  double2* su = sm;
  double2* sT = sm + n2;
  double2* sa = sm + 2 * n2;
  double2* sb = sa + 64;
  const double* M = cls_M + cls_Moff[c];
  const double* xq = qx + cls_qoff[c];
  const double* wq = qw + cls_qoff[c];
  const double* N = qN + cls_qoff[c] * 64;
  const double X0 = ox[e], Y0 = oy[e], HX = hx[e], HY = hy[e];
  const int64_t base = dof_off[e];
  for (int t = threadIdx.x; t < n2; t += NT) su[t] = U[base + t];
  for (int m = threadIdx.x; m < 2 * n; m += NT) {
    const bool yd = m >= n;
    const int mm = yd ? m - n : m;
    double sx = 0, sy = 0;
    for (int t = 0; t < q; ++t) {
      double pos = yd ? Y0 + (xq[t] + 1) * HY / 2 : X0 + (xq[t] + 1) * HX / 2;
      double ph = k * (yd ? dy : dx) * pos;
      double wn = wq[t] * N[(int64_t)t * 64 + mm];
      sx += wn * cos(ph);
      sy += wn * sin(ph);
    }
    if (yd) sb[mm] = make_double2(sx, sy); else sa[mm] = make_double2(sx, sy);
  }
  __syncthreads();
  // T = U M^T (U[c][d] = u[c + n d])
  for (int t = threadIdx.x; t < n2; t += NT) {
    const int cc = t % n, b = t / n;
    double ax = 0, ay = 0;
    for (int dd = 0; dd < n; ++dd) {
      const double m = M[b + n * dd];
      ax += m * su[cc + n * dd].x;
      ay += m * su[cc + n * dd].y;
    }
    sT[t] = make_double2(ax, ay);
  }
  __syncthreads();
  const double f0 = k * k * (HX / 2) * (HY / 2);
  const double fm = k * k * (HX * HY / 4);
  double vx = 0, vy = 0;
  for (int t = threadIdx.x; t < n2; t += NT) {
    const int a = t % n, b = t / n;
    double wx = 0, wy = 0;   // (M U M^T)[a][b]
    for (int cc = 0; cc < n; ++cc) {
      const double m = M[a + n * cc];
      wx += m * sT[cc + n * b].x;
      wy += m * sT[cc + n * b].y;
    }
    const double2 l = Lam[base + t];
    const double2 db = cmul(sa[a], sb[b]);
    double2 mw = make_double2(wx, wy);
    if (mass_fac) mw = cmul(mass_fac[e], mw);   // layers: the mass term carries s_x s_y
    const double px = f0 * db.x + fm * mw.x, py = f0 * db.y + fm * mw.y;
    vx += l.x * px - l.y * py;
    vy += l.x * py + l.y * px;
  }
  red[threadIdx.x] = make_double2(vx, vy);
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      red[threadIdx.x].x += red[threadIdx.x + off].x;
      red[threadIdx.x].y += red[threadIdx.x + off].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[e] = 2.0 * (E.x * red[0].x + E.y * red[0].y);
}

__global__ void k_fill_zero(double2* __restrict__ x, int64_t count) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) x[idx] = make_double2(0.0, 0.0);
}

// Scatter packed element blocks into a zeroed full-element array.
__global__ void k_block_scatter(const int* __restrict__ elems, const int64_t* __restrict__ src_off,
                                const int64_t* __restrict__ dof_off, const double2* __restrict__ src,
                                double2* __restrict__ full, int R) {
  const int b = blockIdx.x;
  const int e = elems[b];
  const int64_t len = src_off[b + 1] - src_off[b];
  const double2* sp = src + src_off[b];
  double2* dp = full + dof_off[e] * R;
  for (int64_t t = threadIdx.x; t < len; t += blockDim.x) dp[t] = sp[t];
}

__global__ void k_dense_scatter(const int64_t* __restrict__ idx, const double2* __restrict__ val, int64_t nnz,
                                double2* __restrict__ M) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nnz) M[idx[t]] = val[t];
}

// ---------------------------------------------------------------------------
// Device-resident GMRES.  The iteration index j lives in device memory so every
// launch has a fixed shape; R (RHS count) divides 64 and thread t owns RHS
// column t % R.  nvec = j + 1 Arnoldi vectors take part in an iteration.

// w[row][r] += sign * sum_{i < nvec} V_i[row][r] h[i][r]; when npart is given the
// block also writes the partial squared norms of the updated w (per RHS column).
__global__ void __launch_bounds__(NT) k_mupdate(const double2* __restrict__ V, int64_t vs, const int* __restrict__ jptr,
                                                int jfix, const double2* __restrict__ hc, double2* __restrict__ w,
                                                int n, int R, double sign, double* __restrict__ npart) {
  __shared__ double2 red[NT];
  const int nvec = (jptr ? *jptr : jfix) + 1;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = threadIdx.x % R;   // NT is a multiple of R, so idx % R == threadIdx.x % R
  double nx = 0;
  if (idx < (int64_t)n * R) {
    double ax = 0, ay = 0;
#pragma unroll 4
    for (int i = 0; i < nvec; ++i) {
      double2 a = V[(int64_t)i * vs + idx], b = hc[i * R + r];
      ax += a.x * b.x - a.y * b.y;
      ay += a.x * b.y + a.y * b.x;
    }
    double2 c = w[idx];
    double2 o = make_double2(c.x + sign * ax, c.y + sign * ay);
    w[idx] = o;
    nx = o.x * o.x + o.y * o.y;
  }
  if (npart) {
    double2 t = block_sum_by_rhs(make_double2(nx, 0), R, red);
    if (threadIdx.x < R) npart[blockIdx.x * R + threadIdx.x] = t.x;
  }
}

// The same update for short vectors (few rows x RHS): a workgroup owns 64
// entries and its four waves take every fourth Arnoldi vector, so that the
// chip holds four times as many waves and each lane has fewer loads in a row.
constexpr int UPD_SPLIT_MAX = 1 << 20;   // entries (rows x RHS) up to which the split form is used

__global__ void __launch_bounds__(NT) k_mupdate_split(const double2* __restrict__ V, int64_t vs,
                                                      const int* __restrict__ jptr, int jfix,
                                                      const double2* __restrict__ hc, double2* __restrict__ w, int n,
                                                      int R, double sign, double* __restrict__ npart) {
  __shared__ double2 red[NT / 64][64];
  const int nvec = (jptr ? *jptr : jfix) + 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
  const bool live = idx < (int64_t)n * R;
  const int r = lane % R;   // 64 is a multiple of R
  double ax = 0, ay = 0;
  if (live) {
#pragma unroll 4
    for (int i = wv; i < nvec; i += NT / 64) {
      const double2 a = V[(int64_t)i * vs + idx], b = hc[i * R + r];
      ax += a.x * b.x - a.y * b.y;
      ay += a.x * b.y + a.y * b.x;
    }
  }
  red[wv][lane] = make_double2(ax, ay);
  __syncthreads();
  if (wv == 0) {
    double nx = 0;
    if (live) {
      double sx = 0, sy = 0;
      for (int q = 0; q < NT / 64; ++q) {
        sx += red[q][lane].x;
        sy += red[q][lane].y;
      }
      const double2 c = w[idx];
      const double2 o = make_double2(c.x + sign * sx, c.y + sign * sy);
      w[idx] = o;
      nx = o.x * o.x + o.y * o.y;
    }
    if (npart) {
      for (int off = 32; off >= R && off > 0; off >>= 1) nx += __shfl_xor(nx, off, 64);
      if (lane < R) npart[(int64_t)blockIdx.x * R + lane] = nx;
    }
  }
}

// Partial squared norms of w per block and RHS column.
__global__ void __launch_bounds__(NT) k_norm2_part(const double2* __restrict__ w, int n, int R, double* __restrict__ part) {
  __shared__ double2 red[NT];
  const int r = threadIdx.x % R, rl = threadIdx.x / R, step = NT / R;
  double acc = 0;
  for (int64_t row = (int64_t)blockIdx.x * step + rl; row < n; row += (int64_t)gridDim.x * step) {
    double2 a = w[row * R + r];
    acc += a.x * a.x + a.y * a.y;
  }
  double2 s = block_sum_by_rhs(make_double2(acc, 0), R, red);
  if (threadIdx.x < R) part[blockIdx.x * R + threadIdx.x] = s.x;
}

// nrm[r] = sqrt(sum of partials); out = w / nrm (zero where nrm = 0).  Every
// block reduces the partials itself; block 0 publishes nrm.  out2 (optional)
// receives the same vector.  The destination is V_kry + (j + 1 + dst_shift) * vs
// when jptr is given, else out directly.
// nrm[r] = sqrt(sum_b part[b][r]): one block per RHS column.
__global__ void __launch_bounds__(NT) k_norm_reduce(const double* __restrict__ part, int nblk, int R,
                                                    double* __restrict__ nrm) {
  __shared__ double2 red[NT];
  const int r = blockIdx.x;
  double acc = 0;
  for (int b = threadIdx.x; b < nblk; b += NT) acc += part[(int64_t)b * R + r];
  double2 t = block_sum_by_rhs(make_double2(acc, 0), 1, red);
  if (threadIdx.x == 0) nrm[r] = sqrt(t.x);
}

// out = w / nrm (zero where nrm = 0); out2 (optional) receives the same vector.
// The destination is V_kry + (j + 1) * vs when jptr is given, else out directly.
__global__ void __launch_bounds__(NT) k_normalize(const double2* __restrict__ w, const double* __restrict__ nrm,
                                                  int n, int R, double2* __restrict__ out,
                                                  const int* __restrict__ jptr, int64_t vs,
                                                  double2* __restrict__ out2) {
  __shared__ double inv[64];
  if (threadIdx.x < R) {
    double nv = nrm[threadIdx.x];
    inv[threadIdx.x] = nv > 0 ? 1.0 / nv : 0.0;
  }
  __syncthreads();
  double2* dst = out + (jptr ? (int64_t)(*jptr + 1) * vs : 0);
  for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < (int64_t)n * R; idx += (int64_t)gridDim.x * NT) {
    double f = inv[idx % R];
    double2 a = w[idx];
    double2 o = make_double2(a.x * f, a.y * f);
    dst[idx] = o;
    if (out2) out2[idx] = o;
  }
}

__device__ __forceinline__ double2 shfl_up2(double2 v, int d) {
  return make_double2(__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64));
}

// Column j of the Hessenberg matrix for system r: entries 0..j in hc and the
// subdiagonal entry sub (real, >= 0); the earlier rotations in csl, snl and
// g_j in gj, all in shared memory or registers.  Applies the earlier
// rotations, forms rotation j, updates g and the residual estimate.  Called
// by every thread of the block; xj_sh is block-shared scratch.
//
// The j earlier rotations form a chain: with x_0 = h_0 and h_i the new column,
// rotation i maps (x_i, h_{i+1}) to the rotated entry t_i = c_i x_i + s_i h_{i+1}
// and the carried value x_{i+1} = -conj(s_i) x_i + c_i h_{i+1}.  The carry is a
// first-order affine recurrence, so the first wave resolves it as a prefix scan
// of affine maps (each lane composes a segment of consecutive rotations, the
// segments are combined across lanes in six shuffle steps) instead of a chain
// of j dependent steps on one lane.
__device__ void givens_column(int j, int r, const double2* hc, double sub, const double2* csl, const double2* snl,
                              double2 gj, double2* __restrict__ H, double2* __restrict__ cs, double2* __restrict__ sn,
                              double2* __restrict__ g, const double* __restrict__ beta, int* __restrict__ done,
                              int* __restrict__ iters, double* __restrict__ resid, double tol, int maxvec, int R,
                              double* __restrict__ hist, double2* xj_sh) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int seg = (j + 63) / 64;
    const int s0 = min(j, lane * seg), s1 = min(j, s0 + seg);
    // this lane's segment as one map x -> A x + B
    double2 A = make_double2(1, 0), B = make_double2(0, 0);
    for (int i = s0; i < s1; ++i) {
      const double2 c = csl[i], s = snl[i], hb = hc[i + 1];
      const double2 al = make_double2(-s.x, s.y);   // -conj(s)
      B = cfma(c, hb, cmul(al, B));
      A = cmul(al, A);
    }
    // inclusive scan over the lanes, earlier segments applied first
    for (int d = 1; d < 64; d <<= 1) {
      const double2 Ap = shfl_up2(A, d), Bp = shfl_up2(B, d);
      if (lane >= d) {
        B = cfma(A, Bp, B);
        A = cmul(A, Ap);
      }
    }
    double2 Ae = shfl_up2(A, 1), Be = shfl_up2(B, 1);
    if (lane == 0) {
      Ae = make_double2(1, 0);
      Be = make_double2(0, 0);
    }
    const double2 x0 = hc[0];
    double2 x = cfma(Ae, x0, Be);   // carried value entering this lane's segment
    for (int i = s0; i < s1; ++i) {
      const double2 c = csl[i], s = snl[i], hb = hc[i + 1];
      H[((int64_t)j * maxvec + i) * R + r] = cfma(c, x, cmul(s, hb));
      x = cfma(c, hb, cmul(make_double2(-s.x, s.y), x));
    }
    if (j == 0 && lane == 0) *xj_sh = x0;
    if (j > 0 && s0 < s1 && s1 == j) *xj_sh = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double2 a = *xj_sh, b = make_double2(sub, 0.0);
    double aa = sqrt(a.x * a.x + a.y * a.y), bb = sqrt(b.x * b.x + b.y * b.y);
    double den = sqrt(aa * aa + bb * bb);
    double2 c, s;
    if (den == 0) { c = make_double2(1, 0); s = make_double2(0, 0); }
    else if (aa == 0) { c = make_double2(0, 0); s = make_double2(b.x / den, -b.y / den); }
    else {
      c = make_double2(aa / den, 0);
      double2 ph = make_double2(a.x / aa, a.y / aa);          // a / |a|
      s = make_double2((ph.x * b.x + ph.y * b.y) / den, (ph.y * b.x - ph.x * b.y) / den);  // ph conj(b) / den
    }
    cs[j * R + r] = c;
    sn[j * R + r] = s;
    H[((int64_t)j * maxvec + j) * R + r] =
        make_double2(c.x * a.x + s.x * b.x - s.y * b.y, c.x * a.y + s.x * b.y + s.y * b.x);
    const double2 gn = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    g[(j + 1) * R + r] = gn;
    g[j * R + r] = make_double2(c.x * gj.x, c.x * gj.y);
    double res = sqrt(gn.x * gn.x + gn.y * gn.y) / beta[r];
    resid[r] = res;
    if (hist) hist[(int64_t)(j + 1) * R + r] = res;
    iters[r] = j + 1;
    if (res <= tol || sub == 0.0) done[r] = 1;
  }
}

// End of an iteration's scalar step: the last block to finish publishes
// status = {all converged, jnext} and sets j = jnext.  The status goes to
// host-mapped coherent memory (slot jnext - 1 mod STATUS_SLOTS), so the host
// reads it without a copy in the stream.
__device__ void publish_step(int jnext, int* __restrict__ jptr, const int* __restrict__ done, int R,
                             int* __restrict__ counter, int* __restrict__ status) {
  __syncthreads();
  int* st = status + 2 * ((jnext - 1) % STATUS_SLOTS);
  if (threadIdx.x == 0 && gridDim.x == 1) {
    // a single system: no other block to wait for (device-wide fences are costly
    // across the chip's separate L2 caches)
    st[0] = done[0];
    st[1] = jnext;
    *jptr = jnext;
  } else if (threadIdx.x == 0) {
    __threadfence();
    int prev = atomicAdd(counter, 1);
    if (prev == gridDim.x - 1) {
      __threadfence();
      int all = 1;
      for (int q = 0; q < R; ++q) all &= __hip_atomic_load(done + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st[0] = all;
      st[1] = jnext;
      *jptr = jnext;
      *counter = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Arnoldi with delayed reorthogonalisation (one multi-dot and one update per
// iteration).  At iteration j the basis q_0..q_{j-1} is final and V_j holds a
// tentative vector u (projected once, scaled); z = P^-1 F u has just been
// formed.  One pass over the basis gives s = Q^H u, t = Q^H z, u^H z, |u|^2 and
// |z|^2, from which
//   q_j   = (u - Q s) / nu,                 nu^2 = |u|^2 - |s|^2,
//   column j-1 of H: h' + rho s on rows 0..j-1 and rho nu on row j, where h'
//          and rho are the first-pass coefficients and scale of u,
//   A q_j = (z - Q_{j+1} H s) / nu, so the first-pass coefficients of column j
//          are ([t; tau] - H s) / nu with tau = q_j^H z = (u^H z - s^H t) / nu,
//   u_next = (z - Q t - q_j tau) / sigma,   sigma^2 = |z|^2 - |t|^2 - |tau|^2,
//          and its scale rho_next = sigma / nu.
// The norms come from the dot products (exact for orthonormal Q); the scale of
// u only has to be the one used, since nu and the column entries are formed
// from the dots of the stored u itself.  Dot entries per chunk: s at 0..j-1, t
// at j..2j-1, then u^H z, |u|^2, |z|^2.

__device__ __forceinline__ void cdot_acc(double2 a, double2 b, double& x, double& y) {  // += conj(a) b
  x += a.x * b.x + a.y * b.y;
  y += a.x * b.y - a.y * b.x;
}

// few right-hand sides: one wave per (row chunk, basis vector or the extra item)
__global__ void __launch_bounds__(NT) k_dmdot_wave(const double2* __restrict__ V, int64_t vs,
                                                   const int* __restrict__ jptr, const double2* __restrict__ z, int n,
                                                   int R, int chunk, int nchunks, int dstride,
                                                   double2* __restrict__ part) {
  const int j = *jptr;
  const int nitems = nchunks * (j + 1);
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (NT / 64);
  const double2* u = V + (int64_t)j * vs;
  for (int item = wave; item < nitems; item += nwaves) {
    const int c = item % nchunks, i = item / nchunks;
    const int64_t lo = (int64_t)c * chunk * R, hi = min((int64_t)n, (int64_t)(c + 1) * chunk) * R;
    double x0 = 0, y0 = 0, x1 = 0, y1 = 0, x2 = 0, y2 = 0;
    if (i < j) {
      const double2* q = V + (int64_t)i * vs;
#pragma unroll 4
      for (int64_t e = lo + lane; e < hi; e += 64) {
        const double2 a = q[e];
        cdot_acc(a, u[e], x0, y0);
        cdot_acc(a, z[e], x1, y1);
      }
    } else {
#pragma unroll 4
      for (int64_t e = lo + lane; e < hi; e += 64) {
        const double2 a = u[e], b = z[e];
        cdot_acc(a, b, x0, y0);
        x1 += a.x * a.x + a.y * a.y;
        x2 += b.x * b.x + b.y * b.y;
      }
    }
    for (int off = 32; off >= R; off >>= 1) {
      x0 += __shfl_xor(x0, off, 64);
      y0 += __shfl_xor(y0, off, 64);
      x1 += __shfl_xor(x1, off, 64);
      y1 += __shfl_xor(y1, off, 64);
      x2 += __shfl_xor(x2, off, 64);
    }
    if (lane < R) {
      double2* pc = part + (int64_t)c * dstride * R + lane;
      if (i < j) {
        pc[(int64_t)i * R] = make_double2(x0, y0);
        pc[(int64_t)(j + i) * R] = make_double2(x1, y1);
      } else {
        pc[(int64_t)(2 * j) * R] = make_double2(x0, y0);
        pc[(int64_t)(2 * j + 1) * R] = make_double2(x1, 0);
        pc[(int64_t)(2 * j + 2) * R] = make_double2(x2, 0);
      }
    }
  }
}

// many right-hand sides: one block per (row chunk, group of DGV basis vectors
// or the extra item), threads own RHS column t % R; grouping the vectors reads
// the long u and z once per group instead of once per vector
constexpr int DGV = 4;

__global__ void __launch_bounds__(NT) k_dmdot_blk(const double2* __restrict__ V, int64_t vs,
                                                  const int* __restrict__ jptr, const double2* __restrict__ z, int n,
                                                  int R, int chunk, int nchunks, int dstride,
                                                  double2* __restrict__ part) {
  __shared__ double2 red[NT];
  const int j = *jptr;
  const int ng = (j + DGV - 1) / DGV;   // vector groups; group ng is the extra item
  const int nitems = nchunks * (ng + 1);
  const int r = threadIdx.x % R, rl = threadIdx.x / R, step = NT / R;
  const double2* u = V + (int64_t)j * vs;
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int c = item % nchunks, gi = item / nchunks;
    const int64_t lo = (int64_t)c * chunk, hi = min((int64_t)n, lo + chunk);
    double2* pc = part + (int64_t)c * dstride * R + r;
    if (gi < ng) {
      const int i0 = gi * DGV;
      double sx[DGV], sy[DGV], tx[DGV], ty[DGV];
#pragma unroll
      for (int t = 0; t < DGV; ++t) sx[t] = sy[t] = tx[t] = ty[t] = 0;
      for (int64_t row = lo + rl; row < hi; row += step) {
        const int64_t o = row * R + r;
        const double2 uo = u[o], zo = z[o];
#pragma unroll
        for (int t = 0; t < DGV; ++t) {
          if (i0 + t < j) {
            const double2 a = V[(int64_t)(i0 + t) * vs + o];
            cdot_acc(a, uo, sx[t], sy[t]);
            cdot_acc(a, zo, tx[t], ty[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < DGV; ++t) {
        if (i0 + t >= j) break;   // uniform over the block
        const double2 s0 = block_sum_by_rhs(make_double2(sx[t], sy[t]), R, red);
        const double2 s1 = block_sum_by_rhs(make_double2(tx[t], ty[t]), R, red);
        if (threadIdx.x < R) {
          pc[(int64_t)(i0 + t) * R] = s0;
          pc[(int64_t)(j + i0 + t) * R] = s1;
        }
      }
    } else {
      double x0 = 0, y0 = 0, x1 = 0, x2 = 0;
      for (int64_t row = lo + rl; row < hi; row += step) {
        const int64_t o = row * R + r;
        const double2 a = u[o], b = z[o];
        cdot_acc(a, b, x0, y0);
        x1 += a.x * a.x + a.y * a.y;
        x2 += b.x * b.x + b.y * b.y;
      }
      const double2 s0 = block_sum_by_rhs(make_double2(x0, y0), R, red);
      const double2 s1 = block_sum_by_rhs(make_double2(x1, x2), R, red);
      if (threadIdx.x < R) {
        pc[(int64_t)(2 * j) * R] = s0;
        pc[(int64_t)(2 * j + 1) * R] = make_double2(s1.x, 0);
        pc[(int64_t)(2 * j + 2) * R] = make_double2(s1.y, 0);
      }
    }
  }
}

// D[k][r] = sum_c part[c][k][r] for k < 2j + 3: one wave per (k, r)
__global__ void __launch_bounds__(NT) k_dmdot_reduce(const double2* __restrict__ part, int nchunks,
                                                     const int* __restrict__ jptr, int dstride, int R,
                                                     double2* __restrict__ D) {
  const int j = *jptr;
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);   // k * R + r
  if (idx >= (2 * j + 3) * R) return;
  double ax = 0, ay = 0;
  for (int c = lane; c < nchunks; c += 64) {
    const double2 a = part[(int64_t)c * dstride * R + idx];
    ax += a.x;
    ay += a.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    ax += __shfl_xor(ax, off, 64);
    ay += __shfl_xor(ay, off, 64);
  }
  if (lane == 0) D[idx] = make_double2(ax, ay);
}

// block-wide sum of (x, y) over all threads; valid in every thread
__device__ __forceinline__ double2 block_sum_all(double x, double y, double2* red) {
  for (int off = 32; off > 0; off >>= 1) {
    x += __shfl_xor(x, off, 64);
    y += __shfl_xor(y, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = make_double2(x, y);
  __syncthreads();
  double2 t = make_double2(0, 0);
  for (int q = 0; q < NT / 64; ++q) {
    t.x += red[q].x;
    t.y += red[q].y;
  }
  return t;
}

// The scalar step of an iteration, one block per system r: finishes column j-1
// of H (stored unrotated in Hraw, then rotated by givens_column), forms the
// update coefficients uc = [s (j), t (j), tau, 1/nu, 1/sigma] and advances j.
// The first-pass coefficients of column j, which need H s, are formed by the
// update kernel that follows (they are first used in the next scalar step).
// Every global value the step needs is loaded up front; the column and the
// earlier rotations are kept in shared memory ((3 maxvec + 1) entries).
__global__ void __launch_bounds__(NT) k_dcgs_scalar(int* __restrict__ jptr, const double2* __restrict__ D,
                                                    double2* __restrict__ Hraw, const double2* __restrict__ hprev,
                                                    double* __restrict__ rho, double2* __restrict__ uc,
                                                    double2* __restrict__ H, double2* __restrict__ cs,
                                                    double2* __restrict__ sn, double2* __restrict__ g,
                                                    const double* __restrict__ beta, int* __restrict__ done,
                                                    int* __restrict__ iters, double* __restrict__ resid, double tol,
                                                    int maxvec, int R, int* __restrict__ counter,
                                                    int* __restrict__ status, double* __restrict__ hist) {
  extern __shared__ double2 shm[];
  double2* col = shm;                  // column j-1: maxvec + 1 entries
  double2* csl = col + maxvec + 1;     // rotations 0..j-2
  double2* snl = csl + maxvec;
  __shared__ double2 red[NT / 64];
  __shared__ double2 xj_sh;
  const int r = blockIdx.x;
  const int j = *jptr;
  const double rho_prev = rho[r];
  const int is_done = done[r];
  const double2 gj = j >= 1 ? g[(j - 1) * R + r] : make_double2(0, 0);
  const double2 uz = D[(int64_t)(2 * j) * R + r];
  const double uu = D[(int64_t)(2 * j + 1) * R + r].x, zz = D[(int64_t)(2 * j + 2) * R + r].x;
  double ss = 0, tt = 0, stx = 0, sty = 0;
  for (int i = threadIdx.x; i < j; i += NT) {
    const double2 a = D[(int64_t)i * R + r], b = D[(int64_t)(j + i) * R + r];
    const double2 hp = hprev[(int64_t)i * R + r];
    if (i < j - 1) {
      csl[i] = cs[(int64_t)i * R + r];
      snl[i] = sn[(int64_t)i * R + r];
    }
    uc[(int64_t)i * R + r] = a;
    uc[(int64_t)(j + i) * R + r] = b;
    col[i] = make_double2(hp.x + rho_prev * a.x, hp.y + rho_prev * a.y);
    ss += a.x * a.x + a.y * a.y;
    tt += b.x * b.x + b.y * b.y;
    cdot_acc(a, b, stx, sty);   // s^H t
  }
  const double2 sum_ss_tt = block_sum_all(ss, tt, red);
  const double2 st = block_sum_all(stx, sty, red);
  const double nu2 = uu - sum_ss_tt.x;
  const double nu = nu2 > 0 ? sqrt(nu2) : 0.0;
  const double inu = nu > 0 ? 1.0 / nu : 0.0;
  if (j >= 1) {
    // column j-1, unrotated, to Hraw (rows 0..j), then rotated
    if (threadIdx.x == 0) col[j] = make_double2(rho_prev * nu, 0);
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += NT) Hraw[((int64_t)(j - 1) * maxvec + i) * R + r] = col[i];
    if (!is_done) givens_column(j - 1, r, col, rho_prev * nu, csl, snl, gj, H, cs, sn, g, beta, done, iters, resid,
                                tol, maxvec, R, hist, &xj_sh);
  }
  if (threadIdx.x == 0) {
    // tau = (u^H z - s^H t) / nu; sigma^2 = |z|^2 - |t|^2 - |tau|^2
    const double2 tau = make_double2((uz.x - st.x) * inu, (uz.y - st.y) * inu);
    const double sg2 = zz - sum_ss_tt.y - (tau.x * tau.x + tau.y * tau.y);
    const double sg = sg2 > 0 ? sqrt(sg2) : 0.0;
    const double isg = sg > 0 ? 1.0 / sg : 0.0;
    uc[(int64_t)(2 * j) * R + r] = tau;
    uc[(int64_t)(2 * j + 1) * R + r] = make_double2(inu, 0);
    uc[(int64_t)(2 * j + 2) * R + r] = make_double2(isg, 0);
    rho[r] = sg * inu;
  }
  publish_step(j + 1, jptr, done, R, counter, status);
}

// First-pass coefficients of column j, hprev = ([t; tau] - H s) / nu with H the
// unrotated (j+1) x j Hessenberg matrix: one (row, system) item per block in
// turn, a block-wide dot over the row.  Every block of the update kernels
// takes part, so that the rows cost no launch of their own.
__device__ void first_pass_rows(int j, int R, int maxvec, const double2* __restrict__ Hraw,
                                const double2* __restrict__ uc, double2* __restrict__ hprev, double2* red) {
  for (int item = blockIdx.x; item < (j + 1) * R; item += gridDim.x) {
    const int i = item / R, r = item - i * R;
    double x = 0, y = 0;
    for (int k = max(0, i - 1) + (int)threadIdx.x; k < j; k += NT) {
      const double2 a = Hraw[((int64_t)k * maxvec + i) * R + r], b = uc[(int64_t)k * R + r];
      x += a.x * b.x - a.y * b.y;
      y += a.x * b.y + a.y * b.x;
    }
    const double2 hs = block_sum_all(x, y, red);
    if (threadIdx.x == 0) {
      const double2 c = uc[(int64_t)(i < j ? j + i : 2 * j) * R + r];
      const double inu = uc[(int64_t)(2 * j + 1) * R + r].x;
      hprev[(int64_t)i * R + r] = make_double2((c.x - hs.x) * inu, (c.y - hs.y) * inu);
    }
  }
}

// The update of iteration j (read as *jptr - 1, after the scalar step):
// V_j = q_j = (u - Q s) / nu and V_{j+1} = out2 = (z - Q t - q_j tau) / sigma.
// Short vectors: a workgroup owns 64 entries and its four waves take every
// fourth basis vector.
__global__ void __launch_bounds__(NT) k_dupdate_split(double2* __restrict__ V, int64_t vs,
                                                      const int* __restrict__ jptr, const double2* __restrict__ uc,
                                                      double2* __restrict__ z, int n, int R,
                                                      double2* __restrict__ out2, const double2* __restrict__ Hraw,
                                                      double2* __restrict__ hprev, int maxvec) {
  __shared__ double2 red[2][NT / 64][64];
  __shared__ double2 red1[NT / 64];
  const int j = *jptr - 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
  const bool live = idx < (int64_t)n * R;
  const int r = lane % R;   // 64 is a multiple of R
  double sx = 0, sy = 0, tx = 0, ty = 0;
  if (live) {
#pragma unroll 4
    for (int i = wv; i < j; i += NT / 64) {
      const double2 a = V[(int64_t)i * vs + idx], b = uc[(int64_t)i * R + r], c = uc[(int64_t)(j + i) * R + r];
      sx += a.x * b.x - a.y * b.y;
      sy += a.x * b.y + a.y * b.x;
      tx += a.x * c.x - a.y * c.y;
      ty += a.x * c.y + a.y * c.x;
    }
  }
  red[0][wv][lane] = make_double2(sx, sy);
  red[1][wv][lane] = make_double2(tx, ty);
  __syncthreads();
  if (wv == 0 && live) {
    double ax = 0, ay = 0, bx = 0, by = 0;
    for (int q = 0; q < NT / 64; ++q) {
      ax += red[0][q][lane].x;
      ay += red[0][q][lane].y;
      bx += red[1][q][lane].x;
      by += red[1][q][lane].y;
    }
    const double2 tau = uc[(int64_t)(2 * j) * R + r];
    const double inu = uc[(int64_t)(2 * j + 1) * R + r].x, isg = uc[(int64_t)(2 * j + 2) * R + r].x;
    const double2 u = V[(int64_t)j * vs + idx], zv = z[idx];
    const double2 q = make_double2((u.x - ax) * inu, (u.y - ay) * inu);
    const double2 un = make_double2((zv.x - bx - (q.x * tau.x - q.y * tau.y)) * isg,
                                    (zv.y - by - (q.x * tau.y + q.y * tau.x)) * isg);
    V[(int64_t)j * vs + idx] = q;
    V[(int64_t)(j + 1) * vs + idx] = un;
    if (out2) out2[idx] = un;
    z[idx] = make_double2(0, 0);   // cleared for the next operator output (added into)
  }
  first_pass_rows(j, R, maxvec, Hraw, uc, hprev, red1);
}

// the same for long vectors: one thread per entry over all basis vectors
__global__ void __launch_bounds__(NT) k_dupdate(double2* __restrict__ V, int64_t vs, const int* __restrict__ jptr,
                                                const double2* __restrict__ uc, double2* __restrict__ z, int n,
                                                int R, double2* __restrict__ out2, const double2* __restrict__ Hraw,
                                                double2* __restrict__ hprev, int maxvec) {
  __shared__ double2 red1[NT / 64];
  const int j = *jptr - 1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)n * R) {
    const int r = threadIdx.x % R;   // NT is a multiple of R
    double ax = 0, ay = 0, bx = 0, by = 0;
#pragma unroll 4
    for (int i = 0; i < j; ++i) {
      const double2 a = V[(int64_t)i * vs + idx], b = uc[(int64_t)i * R + r], c = uc[(int64_t)(j + i) * R + r];
      ax += a.x * b.x - a.y * b.y;
      ay += a.x * b.y + a.y * b.x;
      bx += a.x * c.x - a.y * c.y;
      by += a.x * c.y + a.y * c.x;
    }
    const double2 tau = uc[(int64_t)(2 * j) * R + r];
    const double inu = uc[(int64_t)(2 * j + 1) * R + r].x, isg = uc[(int64_t)(2 * j + 2) * R + r].x;
    const double2 u = V[(int64_t)j * vs + idx], zv = z[idx];
    const double2 q = make_double2((u.x - ax) * inu, (u.y - ay) * inu);
    const double2 un = make_double2((zv.x - bx - (q.x * tau.x - q.y * tau.y)) * isg,
                                    (zv.y - by - (q.x * tau.y + q.y * tau.x)) * isg);
    V[(int64_t)j * vs + idx] = q;
    V[(int64_t)(j + 1) * vs + idx] = un;
    if (out2) out2[idx] = un;
    z[idx] = make_double2(0, 0);
  }
  first_pass_rows(j, R, maxvec, Hraw, uc, hprev, red1);
}

// Start of a GMRES run: g_0 = beta = ||P^-1 rhs||, flags cleared, j = 0.
__global__ void k_gmres_init(const double* __restrict__ nrm, double* __restrict__ beta, double2* __restrict__ g,
                             int* __restrict__ done, int* __restrict__ iters, double* __restrict__ resid,
                             int* __restrict__ jptr, int* __restrict__ counter, int* __restrict__ status, int R,
                             double* __restrict__ hist) {
  int r = threadIdx.x;
  if (r < R) {
    double b = nrm[r];
    beta[r] = b;
    g[r] = make_double2(b, 0);
    done[r] = b > 0 ? 0 : 1;
    iters[r] = 0;
    resid[r] = b > 0 ? 1.0 : 0.0;
    if (hist) hist[r] = resid[r];
  }
  if (r == 0) {
    *jptr = 0;
    *counter = 0;
    status[0] = 0;
    status[1] = 0;
  }
}

inline unsigned nblocks(int64_t n, int t = NT) { return unsigned((n + t - 1) / t); }
inline int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace

// ---------------------------------------------------------------------------
// shared memory of the matrix-core slot kernels at R columns, or 0 when they do
// not apply (R not 16, 32 or 64, or an element's operand or output rows do not
// fit: at most 64 KB and 16 output tiles per element)

// columns per block of the matrix-core slot operators: the handle's choice
// (16, 32 or 64; 32 unless tuned), at most R
static int slot_rb(const Handle& h, int R) { return std::min(R, h.slot_rb); }

static size_t slot_mfma_lds(const Handle& h, int R, int mode) {
  if (R < 16 || R % 16 != 0) return 0;
  const int rb = slot_rb(h, R);
  int rows = 0;   // operand and output rows: m + nr (interface operator) or max(m, nr)
  for (auto& C : h.classes) rows = std::max(rows, mode == 0 ? C.m + C.nr : std::max(C.m, C.nr));
  const size_t lds = size_t(rows) * rb * sizeof(double2);
  if (lds > SLOT_MF_LDS || ((rows + 15) / 16) * (rb / 16) > 16) return 0;
  return lds;
}

bool slot_rows_fused(const Handle& h, int R) { return !h.nonconforming && R < 16; }

void launch_slot_apply_rows(const Handle& h, const double2* v, double2* out, int R, hipStream_t s) {
  const auto& d = h.d;
  hipLaunchKernelGGL(k_slot_apply_rows, dim3(h.E, (R + RC - 1) / RC), dim3(NT), 0, s, d.slot_blk, d.slot_in[2],
                     d.slot_out, d.se, v, out, R);
  HIPCHECK(hipGetLastError());
}

template <class T2>
void launch_slot_apply(const Handle& h, int mode, const T2* v, T2* X, T2* GL, int R, hipStream_t s) {
  dim3 grid(h.E, (R + RC - 1) / RC);
  const auto& d = h.d;
  if constexpr (std::is_same<T2, double2>::value) {
    if (const size_t lds = slot_mfma_lds(h, R, mode)) {
      const int rb = slot_rb(h, R);
      const dim3 g(h.E, R / rb);
#define HDP_MF_ARGS d.slot_blk, d.slot_in[mode], d.op1, d.se, d.phi, d.t_ptr, d.t_dof, d.t_coef, v, nullptr, X, GL, R, rb
      if (mode == 0) hipLaunchKernelGGL(k_slot_mfma<0>, g, dim3(NT), lds, s, HDP_MF_ARGS);
      else if (mode == 1) hipLaunchKernelGGL(k_slot_mfma<1>, g, dim3(NT), lds, s, HDP_MF_ARGS);
      else hipLaunchKernelGGL(k_slot_mfma<2>, g, dim3(NT), lds, s, HDP_MF_ARGS);
#undef HDP_MF_ARGS
      HIPCHECK(hipGetLastError());
      return;
    }
  }
  if constexpr (std::is_same<T2, float2>::value) {
    if (const size_t lds = slot_mfma_lds(h, R, mode)) {   // FP32 operands: half the bytes of the FP64 sizing
      const int rb = slot_rb(h, R);
      const dim3 g(h.E, R / rb);
#define HDP_MF32_ARGS d.slot_blk, d.slot_in[mode], d.op1_f, d.se_f, d.phi_f, d.t_ptr, d.t_dof, d.t_coef, v, nullptr, X, GL, R, rb
      if (mode == 0) hipLaunchKernelGGL((k_slot_mfma32<0, float2>), g, dim3(NT), lds / 2, s, HDP_MF32_ARGS);
      else if (mode == 1) hipLaunchKernelGGL((k_slot_mfma32<1, float2>), g, dim3(NT), lds / 2, s, HDP_MF32_ARGS);
      else hipLaunchKernelGGL((k_slot_mfma32<2, float2>), g, dim3(NT), lds / 2, s, HDP_MF32_ARGS);
#undef HDP_MF32_ARGS
      HIPCHECK(hipGetLastError());
      return;
    }
  }
  const T2* op1;
  const T2* se;
  if constexpr (std::is_same<T2, double2>::value) { op1 = d.op1; se = d.se; }
  else { op1 = d.op1_f; se = d.se_f; }
#define HDP_SLOT_ARGS d.slot_blk, d.slot_in[mode], op1, se, v, X, GL, R
  if (mode == 0)
    hipLaunchKernelGGL((k_slot_apply<T2, 0>), grid, dim3(NT), 0, s, HDP_SLOT_ARGS);
  else if (mode == 1)
    hipLaunchKernelGGL((k_slot_apply<T2, 1>), grid, dim3(NT), 0, s, HDP_SLOT_ARGS);
  else
    hipLaunchKernelGGL((k_slot_apply<T2, 2>), grid, dim3(NT), 0, s, HDP_SLOT_ARGS);
#undef HDP_SLOT_ARGS
  HIPCHECK(hipGetLastError());
}

bool slot_coarse_from_tiles(const Handle& h, int R) {
  return R == 1 && h.coarse_mode == 0 && h.d.Ksym && !h.coarse_refine && !h.nonconforming;
}

template <class T2>
void launch_slot_coarse_sym(const Handle& h, const T2* X, T2* Z, hipStream_t s) {
  const auto& d = h.d;
  const T2* phi;
  if constexpr (std::is_same<T2, double2>::value) phi = d.phi; else phi = d.phi_f;
  int nrmax = 1;
  for (auto& C : h.classes) nrmax = std::max(nrmax, C.nr);
  const size_t shm = size_t(nrmax) * SCP * sizeof(double2);
  hipLaunchKernelGGL((k_slot_coarse_sym<T2>), dim3(h.E), dim3(NT), shm, s, d.slot_blk, phi, d.t_ptr, d.t_dof,
                     d.t_coef, X, d.sym_part, h.sym_nt, Z);
  HIPCHECK(hipGetLastError());
}
template void launch_slot_coarse_sym<double2>(const Handle&, const double2*, double2*, hipStream_t);
template void launch_slot_coarse_sym<float2>(const Handle&, const float2*, float2*, hipStream_t);

template <class T2>
static void slot_coarse_impl(const Handle& h, const T2* X, const double2* w, T2* Z, int R, hipStream_t s,
                             const int* t_ptr, const int* t_dof, const double* t_coef);

template <class T2>
void launch_slot_coarse(const Handle& h, const T2* X, const double2* w, T2* Z, int R, hipStream_t s) {
  slot_coarse_impl(h, X, w, Z, R, s, h.d.t_ptr, h.d.t_dof, h.d.t_coef);
}

void launch_slot_coarse_cm(const Handle& h, const double2* X, const double2* cm, double2* Z, int R, hipStream_t s) {
  slot_coarse_impl(h, X, cm, Z, R, s, h.d.id_ptr, h.d.id_dof, h.d.id_coef);
}

template <class T2>
static void slot_coarse_impl(const Handle& h, const T2* X, const double2* w, T2* Z, int R, hipStream_t s,
                             const int* t_ptr, const int* t_dof, const double* t_coef) {
  dim3 grid(h.E, (R + RC - 1) / RC);
  const auto& d = h.d;
  if constexpr (std::is_same<T2, double2>::value) {
    if (const size_t lds = slot_mfma_lds(h, R, 3)) {
      const int rb = slot_rb(h, R);
      hipLaunchKernelGGL(k_slot_mfma<3>, dim3(h.E, R / rb), dim3(NT), lds, s, d.slot_blk, nullptr, d.op1, d.se,
                         d.phi, t_ptr, t_dof, t_coef, w, X, Z, nullptr, R, rb);
      HIPCHECK(hipGetLastError());
      return;
    }
  }
  if constexpr (std::is_same<T2, float2>::value) {
    if (const size_t lds = slot_mfma_lds(h, R, 3)) {
      const int rb = slot_rb(h, R);
      hipLaunchKernelGGL((k_slot_mfma32<3, double2>), dim3(h.E, R / rb), dim3(NT), lds / 2, s, d.slot_blk, nullptr,
                         d.op1_f, d.se_f, d.phi_f, t_ptr, t_dof, t_coef, w, X, Z, nullptr, R, rb);
      HIPCHECK(hipGetLastError());
      return;
    }
  }
  const T2* phi;
  if constexpr (std::is_same<T2, double2>::value) phi = d.phi; else phi = d.phi_f;
  hipLaunchKernelGGL((k_slot_coarse<T2>), grid, dim3(NT), 0, s, d.slot_blk, phi, t_ptr, t_dof, t_coef, X, w, Z, R);
  HIPCHECK(hipGetLastError());
}

template <class T2>
void launch_rowgather(const Handle& h, const T2* src, bool full, bool precond, const double2* w, double2* u, int R,
                      hipStream_t s) {
  const auto& d = h.d;
  if (!h.nonconforming) w = nullptr;
  hipLaunchKernelGGL((k_rowgather<T2>), dim3(nblocks(int64_t(h.nlam) * R)), dim3(NT), 0, s, h.nlam, d.row_slot,
                     d.row_coef, precond ? d.row_xinv : nullptr, full ? d.slot_pos : nullptr, src, d.c2_ptr,
                     d.c2_dof, d.c2_coef, w, u, R);
  HIPCHECK(hipGetLastError());
}

template <class T2>
void launch_assemble(const Handle& h, const T2* GL, const double2* Bfull, const double2* v, double vsign, double2* g,
                     int R, hipStream_t s) {
  const auto& d = h.d;
  if (!h.nonconforming) v = nullptr;
  if (R == 1 && h.nonconforming) {   // long expansion and C_2 lists on hanging edges
    hipLaunchKernelGGL((k_assemble1<T2>), dim3(nblocks(h.nK, NT / 64)), dim3(NT), 0, s, h.nK, d.cdof_ptr, d.cdof_list,
                       d.cdof_coef, GL, d.cm_pos, Bfull, d.c2t_ptr, d.c2t_row, d.c2t_coef, v, vsign, g);
    HIPCHECK(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL((k_assemble<T2>), dim3(nblocks(int64_t(h.nK) * R)), dim3(NT), 0, s, h.nK, d.cdof_ptr,
                     d.cdof_list, d.cdof_coef, GL, d.cm_pos, Bfull, d.c2t_ptr, d.c2t_row, d.c2t_coef, v, vsign, g,
                     R);
  HIPCHECK(hipGetLastError());
}

void launch_hblock(const Handle& h, bool y2, const double2* x, bool in_gather, const double2* add, double2* y,
                   bool out_scatter, int R, hipStream_t s) {
  const auto& d = h.d;
  if (h.nh == 0) return;
  hipLaunchKernelGGL(k_hblock, dim3(nblocks(h.nh, NT / 64)), dim3(NT), 0, s, h.nh, d.hb_blk, d.hb_off, d.hb_rows,
                     d.hb_moff, y2 ? d.hb_y2 : d.hb_xinv, x, int(in_gather), add, y, int(out_scatter), R);
  HIPCHECK(hipGetLastError());
}

template void launch_slot_apply<double2>(const Handle&, int, const double2*, double2*, double2*, int, hipStream_t);
template void launch_slot_apply<float2>(const Handle&, int, const float2*, float2*, float2*, int, hipStream_t);
template void launch_slot_coarse<double2>(const Handle&, const double2*, const double2*, double2*, int, hipStream_t);
template void launch_slot_coarse<float2>(const Handle&, const float2*, const double2*, float2*, int, hipStream_t);
template void launch_rowgather<double2>(const Handle&, const double2*, bool, bool, const double2*, double2*, int,
                                        hipStream_t);
template void launch_rowgather<float2>(const Handle&, const float2*, bool, bool, const double2*, double2*, int,
                                       hipStream_t);
template void launch_assemble<double2>(const Handle&, const double2*, const double2*, const double2*, double,
                                       double2*, int, hipStream_t);
template void launch_assemble<float2>(const Handle&, const float2*, const double2*, const double2*, double, double2*,
                                      int, hipStream_t);

// Strip sweeps of the block-tridiagonal coarse factor at one column.
void launch_coarse_symv_tiles(const Handle& h, const double2* g, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_symv_tiles, dim3(h.sym_ntiles), dim3(SYM_WAVES * 64), 0, s, h.nK, h.sym_nt,
                     h.d.sym_tij, h.d.Ksym, g, h.d.sym_part);
  HIPCHECK(hipGetLastError());
}

void launch_coarse_symv_reduce(const Handle& h, double2* w, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_symv_reduce, dim3(h.sym_nt), dim3(NT), 0, s, h.nK, h.sym_nt, h.d.sym_part, w);
  HIPCHECK(hipGetLastError());
}

void launch_coarse_solve(const Handle& h, const double2* g, double2* w, int R, hipStream_t s) {
  if (R == 1 && h.d.Ksym) {
    launch_coarse_symv_tiles(h, g, s);
    launch_coarse_symv_reduce(h, w, s);
    return;
  }
  hipLaunchKernelGGL(k_coarse_gemv, dim3(nblocks(h.nK, NT / 64)), dim3(NT), 0, s, h.nK, h.d.Kinv, g, w, R);
  HIPCHECK(hipGetLastError());
}

int sym_tile_size() { return SYM_TILE; }

void launch_pack_sym_tiles(const Handle& h, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_sym_tiles, dim3(h.sym_ntiles), dim3(NT), 0, s, h.nK, h.d.Kinv, h.d.sym_tij, h.d.Ksym);
  HIPCHECK(hipGetLastError());
}

// right-hand sides per block of the full-element kernels: the largest power of
// two <= R whose two n^2 stages and the three n^2 class operators fit 64 KB of
// shared memory
static int fdm_chunk(const Handle& h, int R, bool staged) {
  int nmax = 0;
  for (auto& C : h.classes) nmax = std::max(nmax, C.n);
  const int extra = staged ? 3 : 0;
  int rch = 1;
  while (rch * 2 <= R && size_t(nmax) * nmax * (2 * (rch * 2) + extra) * sizeof(double2) <= 65536) rch *= 2;
  return rch;
}

void launch_fdm(const Handle& h, const double2* in, double2* out, int R, hipStream_t s, bool zero_coarse,
                const double2* nu) {
  int nmax = 0;
  for (auto& C : h.classes) nmax = std::max(nmax, C.n);
  const bool staged = size_t(nmax) * nmax * 5 * sizeof(double2) <= 65536;
  const int rch = fdm_chunk(h, R, staged);
  const size_t shm = size_t(nmax) * nmax * (2 * rch + (staged ? 3 : 0)) * sizeof(double2);
  const auto& d = h.d;
  const dim3 grid(h.E, (R + rch - 1) / rch);
  const int zc = zero_coarse ? 1 : 0;
  if (staged)
    hipLaunchKernelGGL(k_fdm<true>, grid, dim3(NT), shm, s, d.elem_cls, d.dof_off, d.cls_n, d.cls_E, d.cls_D, d.Ex,
                       d.Ey, d.Dinv, in, out, R, rch, d.cls_nr, d.cls_R, d.r_modes, zc, d.slot_off, d.slot_pos,
                       d.slot_row, d.slot_coef, zero_coarse ? nu : nullptr);
  else
    hipLaunchKernelGGL(k_fdm<false>, grid, dim3(NT), shm, s, d.elem_cls, d.dof_off, d.cls_n, d.cls_E, d.cls_D, d.Ex,
                       d.Ey, d.Dinv, in, out, R, rch, d.cls_nr, d.cls_R, d.r_modes, zc, d.slot_off, d.slot_pos,
                       d.slot_row, d.slot_coef, zero_coarse ? nu : nullptr);
  HIPCHECK(hipGetLastError());
}

static size_t fdm_mf_lds(const Handle& h, int rc, bool coarse);

// Matrix-core element solves: classes of at most 32 modes per direction, and
// (coarse: the two passes, which keep K_e in shared memory) one column's
// shared memory within the 160 KiB of a compute unit.
bool fdm_mf_ok(const Handle& h, bool coarse) {
  for (auto& C : h.classes)
    if (C.n > 32) return false;
  return fdm_mf_lds(h, 1, coarse) <= 160 * 1024;
}

static int fdm_npmax(const Handle& h) {
  int nmax = 1;
  for (auto& C : h.classes) nmax = std::max(nmax, C.n);
  return nmax <= 16 ? 16 : 32;
}

static int fdm_nrmax(const Handle& h) {
  int nrmax = 1;
  for (auto& C : h.classes) nrmax = std::max(nrmax, C.nr);
  return nrmax;
}

static int fdm_nmax(const Handle& h) {
  int nmax = 1;
  for (auto& C : h.classes) nmax = std::max(nmax, C.n);
  return nmax;
}

static size_t fdm_mf_lds(const Handle& h, int rc, bool coarse) {
  return fdm_mf_entries(fdm_nmax(h), fdm_npmax(h), fdm_nrmax(h), rc, coarse) * sizeof(double2);
}

// Columns per block: the autotuned or requested choice when one is set, else
// the largest power of two up to 8 (and up to R) whose shared memory stays
// within 80 KiB (two blocks per compute unit).
int fdm_mf_rc(const Handle& h, int R) {
  const int cap = std::min(16, pow2_at_least(R));
  const bool coarse = fdm_mf_ok(h, true);
  if (h.fdm_rc > 0 && h.fdm_rc <= cap && fdm_mf_lds(h, h.fdm_rc, coarse) <= 160 * 1024) return h.fdm_rc;
  int rc = 1;
  while (rc * 2 <= std::min(cap, 8) && fdm_mf_lds(h, rc * 2, coarse) <= 80 * 1024) rc *= 2;
  return rc;
}

void launch_coarse_minus_tw(const Handle& h, const double2* w, int R, hipStream_t s) {
  const auto& d = h.d;
  hipLaunchKernelGGL(k_coarse_minus_tw, dim3(nblocks(int64_t(h.ncm) * R)), dim3(NT), 0, s, h.ncm, R, d.t_ptr, d.t_dof,
                     d.t_coef, w, d.cmX, 0);
  HIPCHECK(hipGetLastError());
}

void launch_fdm_mf(const Handle& h, int mode, const double2* in, double2* out, int R, hipStream_t s,
                   const double2* nu, const double2* w, int rc, const double2* kx, double2* xslot) {
  const int np = fdm_npmax(h), nrmax = fdm_nrmax(h), nmax = fdm_nmax(h);
  if (!fdm_mf_ok(h, mode != 0)) fail(HDP_E_UNSUPPORTED, "matrix-core element solve: class too large");
  if (rc <= 0) rc = fdm_mf_rc(h, R);
  const size_t shm = fdm_mf_lds(h, rc, mode != 0);
  if (shm > 160 * 1024) rc = 1;
  const size_t shm1 = fdm_mf_lds(h, rc, mode != 0);
  if (shm1 > 160 * 1024) fail(HDP_E_UNSUPPORTED, "matrix-core element solve: shared memory exceeded");
  const auto& d = h.d;
  if (mode == 2) {   // x_R - T_e w in place, before the corrected solve
    hipLaunchKernelGGL(k_coarse_minus_tw, dim3(nblocks(int64_t(h.ncm) * R)), dim3(NT), 0, s, h.ncm, R, d.t_ptr,
                       d.t_dof, d.t_coef, w, d.cmX, kx ? 1 : 0);
    HIPCHECK(hipGetLastError());
  }
  FdmArgs a{d.fdm_rec, d.order, d.elem_cls, d.dof_off, d.cls_n, d.cls_E, d.cls_D, d.Ex, d.Ey, d.Dinv, d.cls_real, in, out, R,
            d.cls_nr, d.cls_R, d.r_modes, mode != 0 ? 1 : 0, d.slot_off, d.slot_pos, d.slot_row, d.slot_coef,
            mode != 0 ? nu : nullptr, d.cm_off, d.cls_Kc, d.Kc, d.cmX, d.cmA, d.t_ptr, d.t_dof, d.t_coef, w,
            mode == 2 ? kx : nullptr, mode == 1 ? xslot : nullptr};
  const int nchunk = (R + rc - 1) / rc, nitems = h.E * nchunk;
  // blocks resident at once: shared memory and 3 waves per SIMD allow this many per compute unit
  const int per_cu = std::max(1, std::min(3, int((160 * 1024) / shm1)));
  const dim3 grid(std::min(nitems, 256 * per_cu));
#define HDP_FDM_LAUNCH(RCV, NPV)                                                                                 \
  if (mode == 0) hipLaunchKernelGGL((k_fdm_mf<RCV, 0, NPV>), grid, dim3(NT), shm1, s, a, nmax, nrmax, nitems, nchunk);  \
  else if (mode == 1)                                                                                            \
    hipLaunchKernelGGL((k_fdm_mf<RCV, 1, NPV>), grid, dim3(NT), shm1, s, a, nmax, nrmax, nitems, nchunk);               \
  else hipLaunchKernelGGL((k_fdm_mf<RCV, 2, NPV>), grid, dim3(NT), shm1, s, a, nmax, nrmax, nitems, nchunk);
#define HDP_FDM_CASE(RCV)            \
  case RCV:                          \
    if (np == 16) {                  \
      HDP_FDM_LAUNCH(RCV, 16)        \
    } else {                         \
      HDP_FDM_LAUNCH(RCV, 32)        \
    }                                \
    break;
  switch (rc) {
    HDP_FDM_CASE(1)
    HDP_FDM_CASE(2)
    HDP_FDM_CASE(4)
    HDP_FDM_CASE(8)
    HDP_FDM_CASE(16)
    default: fail(HDP_E_ARG, "element solve: columns per block must be 1, 2, 4, 8 or 16");
  }
#undef HDP_FDM_CASE
#undef HDP_FDM_LAUNCH
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
  const int rch = std::min(fdm_chunk(h, R, false), 8);
  const size_t shm = size_t(2) * NRMAX * rch * sizeof(double2);
  hipLaunchKernelGGL(k_correct, dim3(h.E, (R + rch - 1) / rch), dim3(NT), shm, s, d.elem_cls, d.dof_off, d.cm_off,
                     d.cls_n, d.cls_nr, d.cls_R, d.r_modes, d.cls_Kc, d.Kc, d.cls_G, d.G, d.t_ptr, d.t_dof, d.t_coef, X,
                     w, R, rch);
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

GmresDims gmres_dims(int n, int R, int maxvec) {
  GmresDims g;
  g.step = NT / R;
  g.wave = R < 8;
  g.ngroups = maxvec;   // one basis vector per multi-dot item
  if (g.wave) {
    // one wave per (chunk, basis vector): 256 entries per chunk (four per lane),
    // more when the partial buffer's 512 chunks would not cover the rows; a
    // grid of up to 4,096 workgroups (16,384 waves) strides over the items
    g.chunk = int(std::max<int64_t>(256 / R, (int64_t(n) + 511) / 512));
    g.nchunks = int((int64_t(n) + g.chunk - 1) / g.chunk);
    g.grid = int(std::max<int64_t>(1, std::min<int64_t>(4096, (int64_t(g.nchunks) * g.ngroups + 3) / 4)));
  } else {
    // up to 512 row chunks (the partial buffer holds 512) keep the chip busy with
    // many right-hand sides while only a few Arnoldi vectors exist
    g.chunk = int(std::max<int64_t>(g.step, (int64_t(n) + 511) / 512));
    g.nchunks = int((int64_t(n) + g.chunk - 1) / g.chunk);
    g.grid = int(std::max<int64_t>(1, std::min<int64_t>(2048, int64_t(g.nchunks) * ((maxvec + DGV - 1) / DGV + 1))));
  }
  g.nnorm = int(std::max<int64_t>(1, std::min<int64_t>(256, (int64_t(n) * R + NT - 1) / NT)));
  return g;
}

void launch_mupdate(const double2* V, int64_t vs, const int* jptr, int jfix, const double2* hc, double2* w, int n,
                    int R, double sign, double* npart, hipStream_t s) {
  if (int64_t(n) * R <= UPD_SPLIT_MAX)
    hipLaunchKernelGGL(k_mupdate_split, dim3(nblocks(int64_t(n) * R, 64)), dim3(NT), 0, s, V, vs, jptr, jfix, hc, w, n,
                       R, sign, npart);
  else
    hipLaunchKernelGGL(k_mupdate, dim3(nblocks(int64_t(n) * R)), dim3(NT), 0, s, V, vs, jptr, jfix, hc, w, n, R, sign,
                       npart);
  HIPCHECK(hipGetLastError());
}

void launch_normalize(const double2* w, int n, int R, const GmresDims& g, double* part, double* nrm, double2* out,
                      const int* jptr, int64_t vs, double2* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2_part, dim3(g.nnorm), dim3(NT), 0, s, w, n, R, part);
  hipLaunchKernelGGL(k_norm_reduce, dim3(R), dim3(NT), 0, s, part, g.nnorm, R, nrm);
  hipLaunchKernelGGL(k_normalize, dim3(g.nnorm), dim3(NT), 0, s, w, nrm, n, R, out, jptr, vs, out2);
  HIPCHECK(hipGetLastError());
}

void launch_dmdot(const double2* V, int64_t vs, const int* jptr, const double2* z, int n, int R, const GmresDims& g,
                  int dstride, double2* part, hipStream_t s) {
  if (g.wave)
    hipLaunchKernelGGL(k_dmdot_wave, dim3(g.grid), dim3(NT), 0, s, V, vs, jptr, z, n, R, g.chunk, g.nchunks, dstride,
                       part);
  else
    hipLaunchKernelGGL(k_dmdot_blk, dim3(g.grid), dim3(NT), 0, s, V, vs, jptr, z, n, R, g.chunk, g.nchunks, dstride,
                       part);
  HIPCHECK(hipGetLastError());
}

void launch_dmdot_reduce(const double2* part, const GmresDims& g, const int* jptr, int dstride, int R, double2* D,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_dmdot_reduce, dim3(nblocks(int64_t(dstride) * R, NT / 64)), dim3(NT), 0, s, part, g.nchunks,
                     jptr, dstride, R, D);
  HIPCHECK(hipGetLastError());
}

void launch_dcgs_scalar(int* jptr, const double2* D, double2* Hraw, const double2* hprev, double* rho, double2* uc,
                        double2* H, double2* cs, double2* sn, double2* g, const double* beta, int* done, int* iters,
                        double* resid, double tol, int maxvec, int R, int* counter, int* status, double* hist,
                        hipStream_t s) {
  const size_t shm = (3 * size_t(maxvec) + 1) * sizeof(double2);
  hipLaunchKernelGGL(k_dcgs_scalar, dim3(R), dim3(NT), shm, s, jptr, D, Hraw, hprev, rho, uc, H, cs, sn, g, beta,
                     done, iters, resid, tol, maxvec, R, counter, status, hist);
  HIPCHECK(hipGetLastError());
}

void launch_dupdate(double2* V, int64_t vs, const int* jptr, const double2* uc, double2* z, int n, int R,
                    double2* out2, const double2* Hraw, double2* hprev, int maxvec, hipStream_t s) {
  if (int64_t(n) * R <= UPD_SPLIT_MAX)
    hipLaunchKernelGGL(k_dupdate_split, dim3(nblocks(int64_t(n) * R, 64)), dim3(NT), 0, s, V, vs, jptr, uc, z, n, R,
                       out2, Hraw, hprev, maxvec);
  else
    hipLaunchKernelGGL(k_dupdate, dim3(nblocks(int64_t(n) * R)), dim3(NT), 0, s, V, vs, jptr, uc, z, n, R, out2, Hraw,
                       hprev, maxvec);
  HIPCHECK(hipGetLastError());
}

void launch_gmres_init(const double* nrm, double* beta, double2* g, int* done, int* iters, double* resid, int* jptr,
                       int* counter, int* status, int R, double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(64), 0, s, nrm, beta, g, done, iters, resid, jptr, counter, status,
                     R, hist);
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

void launch_block_scatter(const int* elems, const int64_t* src_off, int nblk, const int64_t* dof_off,
                          const double2* src, double2* full, int R, hipStream_t s) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_block_scatter, dim3(nblk), dim3(NT), 0, s, elems, src_off, dof_off, src, full, R);
  HIPCHECK(hipGetLastError());
}

void launch_far_field(const Handle& h, const double2* X, int R, int nrhs_out, double2* E, hipStream_t s) {
  const auto& d = h.d;
  const auto& f = h.far;
  if (f.nsides == 0) {
    launch_fill_zero(E, int64_t(nrhs_out) * f.nfar, s);
    return;
  }
  hipLaunchKernelGGL(k_far_trace, dim3(f.nsides, R), dim3(NT), 0, s, f.elem, f.side, f.node_off, f.tab_off, f.tab,
                     f.dscale, d.elem_cls, d.cls_n, d.dof_off, X, R, f.U, f.DU);
  hipLaunchKernelGGL(k_far_sum, dim3(f.nfar), dim3(NT), 0, s, f.nq, f.px, f.py, f.pw, f.pnx, f.pny, f.ang, h.k, f.U,
                     f.DU, R, nrhs_out, f.nfar, E);
  HIPCHECK(hipGetLastError());
}

void launch_plane_wave_loads(const Handle& h, int kind, const int* elems, int nel, const double* angles, double2* B,
                             int nrhs, int R, hipStream_t s) {
  if (nel == 0 || nrhs == 0) return;
  if (nrhs > R) fail(HDP_E_ARG, "plane-wave loads: more right-hand sides than the stride");
  const auto& d = h.d;
  hipLaunchKernelGGL(k_plane_wave_loads, dim3(nel, nrhs), dim3(NT), 0, s, kind, elems, d.elem_cls, d.cls_n, d.dof_off,
                     d.cls_q, d.cls_qoff, d.qx, d.qw, d.qN, d.ox, d.oy, d.hx, d.hy, d.eps, d.bmask, angles, h.k, B, R);
  HIPCHECK(hipGetLastError());
}

void launch_eps_gradient(const Handle& h, const double2* U, const double2* Lam, double2 E, double incidence,
                         double* grad, hipStream_t s) {
  const auto& d = h.d;
  int nmax = 0;
  for (auto& C : h.classes) nmax = std::max(nmax, C.n);
  const size_t shm = (size_t(2) * nmax * nmax + 128) * sizeof(double2);
  hipLaunchKernelGGL(k_eps_grad, dim3(h.E), dim3(NT), shm, s, d.elem_cls, d.cls_n, d.dof_off, d.cls_q, d.cls_qoff,
                     d.qx, d.qw, d.qN, d.cls_M, d.cls_Moff, d.ox, d.oy, d.hx, d.hy, d.mass_fac, U, Lam, E, h.k,
                     std::cos(incidence), std::sin(incidence), grad);
  HIPCHECK(hipGetLastError());
}

void launch_fill_zero(double2* x, int64_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3(nblocks(count)), dim3(NT), 0, s, x, count);
  HIPCHECK(hipGetLastError());
}

void launch_nd_fwd1(const ND1Fwd* task, int ntask, const NDView& v, const double2* g, double2* F, double2* A,
                    hipStream_t s) {
  if (ntask == 0) return;
  hipLaunchKernelGGL(k_nd_fwd1, dim3(nblocks(ntask, NT / 64)), dim3(NT), 0, s, task, ntask, v.fac, g, F, A);
  HIPCHECK(hipGetLastError());
}

void launch_nd_bwd1(const ND1Bwd* task, int ntask, const NDView& v, const double2* g, const double2* F, double2* X,
                    hipStream_t s) {
  if (ntask == 0) return;
  hipLaunchKernelGGL(k_nd_bwd1, dim3(nblocks(ntask, NT / 64)), dim3(NT), 0, s, task, ntask, v.fac, v.bnd, g, F, X);
  HIPCHECK(hipGetLastError());
}

void launch_nd_tiles(bool bwd, const int4* task, int ntiles, int S, const NDView& v, const double2* g, double2* X,
                     int R, double2* P, hipStream_t s) {
  if (ntiles == 0) return;
  if (R > v.ld) fail(HDP_E_ARG, "nested-dissection sweep: more columns than the slot stride");
  const NDNodes nd{v.off, v.boff, v.bnd, v.uoff, v.push, v.mD, v.mL, v.mLt, v.fac,
                   v.push2, v.child, v.slot, v.ld, v.srows, v.nK};
  double2* part = S > 1 ? P : nullptr;
  const unsigned nt = unsigned(ntiles) * unsigned(S);
  // 16, 32 or 64 columns go to the matrix cores
  const bool mf = R >= 16 && R % 16 == 0;
  if (bwd) {
    if (mf) hipLaunchKernelGGL(k_nd_bwdR<true>, dim3(nt), dim3(NT), 0, s, task, nd, g, X, R, part);
    else hipLaunchKernelGGL(k_nd_bwdR<false>, dim3(nt), dim3(NT), 0, s, task, nd, g, X, R, part);
  } else {
    if (mf) hipLaunchKernelGGL(k_nd_fwdR<true>, dim3(nt), dim3(NT), 0, s, task, nd, g, R, part);
    else hipLaunchKernelGGL(k_nd_fwdR<false>, dim3(nt), dim3(NT), 0, s, task, nd, g, R, part);
  }
  if (S > 1)
    hipLaunchKernelGGL(k_nd_reduce, dim3(nblocks(int64_t(ntiles) * SMJ * R)), dim3(NT), 0, s, task, ntiles, S, P, nd,
                       X, R, bwd ? 1 : 0);
  HIPCHECK(hipGetLastError());
}

void launch_csr_residual(int n, const int64_t* ptr, const int* col, const double2* val, const double2* x,
                         const double2* g, double2* r, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_csr_residual, dim3(nblocks(n, NT / 64)), dim3(NT), 0, s, n, ptr, col, val, x, g, r, R);
  HIPCHECK(hipGetLastError());
}

void launch_nd_top_gather(int n, const int* idx, const int64_t* gptr, const int* grow, const double2* g,
                          const double2* slot, int64_t ld, int64_t sst, double2* r, int R, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_nd_top_gather, dim3(nblocks(int64_t(n) * R)), dim3(NT), 0, s, n, idx, gptr, grow, g, slot, ld,
                     sst, r, R);
  HIPCHECK(hipGetLastError());
}

void launch_nd_top_scatter(int n, const int* idx, const double2* x, double2* w, int R, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_nd_top_scatter, dim3(nblocks(int64_t(n) * R)), dim3(NT), 0, s, n, idx, x, w, R);
  HIPCHECK(hipGetLastError());
}

void launch_nd_top_collect(int n, const int* idx, const double2* w, int R, int k0, int cols, double2* M,
                           hipStream_t s) {
  if (n == 0 || cols == 0) return;
  hipLaunchKernelGGL(k_nd_top_collect, dim3(nblocks(int64_t(n) * cols)), dim3(NT), 0, s, n, idx, w, R, k0, cols, M);
  HIPCHECK(hipGetLastError());
}

void launch_dense_scatter(const int64_t* idx, const double2* val, int64_t nnz, double2* M, hipStream_t s) {
  if (nnz == 0) return;
  hipLaunchKernelGGL(k_dense_scatter, dim3(nblocks(nnz)), dim3(NT), 0, s, idx, val, nnz, M);
  HIPCHECK(hipGetLastError());
}

}  // namespace hdp
