// Launchers of the device kernels (kernels.hip).  All arrays are device
// pointers; "R" is the right-hand-side stride (RHS index fastest).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hdp {

struct Handle;

// Class-batched boundary operators on dual slots (one block per element).
// mode 0: X = D_c y, GL = Phi_c^T y, with y_s = coef_s v[row_s]            (F, first half)
// mode 1: X = Se y with y_s = coef_s v[row_s] / (C1 C1^T)_row              (P^-1, first half)
// mode 2: as mode 1 with v a dual-slot array z and v[row] = (C_1 z)[row]     (P^-1 F, fused)
// the preconditioner on dual slots with its row gather fused (FP64, R < 16,
// conforming meshes): out must be zero on entry
bool slot_rows_fused(const Handle& h, int R);
void launch_slot_apply_rows(const Handle& h, const double2* v, double2* out, int R, hipStream_t s);
// k_slot_coarse reading the coarse solution from the partial sums of the tiled
// coarse apply (one right-hand side, dense coarse inverse, no refinement,
// conforming mesh): the row-sum kernel is skipped
bool slot_coarse_from_tiles(const Handle& h, int R);
template <class T2>
void launch_slot_coarse_sym(const Handle& h, const T2* X, T2* Z, hipStream_t s);
template <class T2>
void launch_slot_apply(const Handle& h, int mode, const T2* v, T2* X, T2* GL, int R, hipStream_t s);
// Z = X + Phi_c (T_e w)
template <class T2>
void launch_slot_coarse(const Handle& h, const T2* X, const double2* w, T2* Z, int R, hipStream_t s);
// Z = X - Phi_c cm with cm per-element coarse-mode values ([ncm][R], FP64)
void launch_slot_coarse_cm(const Handle& h, const double2* X, const double2* cm, double2* Z, int R, hipStream_t s);
// cmX -= T_e w at every coarse mode
void launch_coarse_minus_tw(const Handle& h, const double2* w, int R, hipStream_t s);
// u[row] = scale_row * (sum coef * src[pos(slot)] + (C_2 w)[row])  (pos = slot if full == false;
// the C_2 term only on meshes with hanging edges and w != nullptr)
template <class T2>
void launch_rowgather(const Handle& h, const T2* src, bool full, bool precond, const double2* w, double2* u, int R,
                      hipStream_t s);
// g = T^T (GL + Bfull at the coarse modes) + vsign C_2^T v   (T: coarse-mode expansions)
template <class T2>
void launch_assemble(const Handle& h, const T2* GL, const double2* Bfull, const double2* v, double vsign, double2* g,
                     int R, hipStream_t s);
// Dense blocks over the hanging dual rows: y = add + M x with M = X^-1 (y2 false) or Y_2;
// x gathered from a dual vector (in_gather) or compact [nh][R]; y scattered or compact
void launch_hblock(const Handle& h, bool y2, const double2* x, bool in_gather, const double2* add, double2* y,
                   bool out_scatter, int R, hipStream_t s);
// w = K^-1 g (dense, FP64)
void launch_coarse_solve(const Handle& h, const double2* g, double2* w, int R, hipStream_t s);

// Full-element operations (arrays [dof][R])
// With zero_coarse the element's coarse-mode entries of `in` are read as zero
// (the solve of the interior problem from a full load vector, out of place);
// with nu ([nlam][R]) the dual slots read in - C^T nu as well.
void launch_fdm(const Handle& h, const double2* in, double2* out, int R, hipStream_t s, bool zero_coarse = false,
                const double2* nu = nullptr);
void launch_zero_R(const Handle& h, double2* X, int R, hipStream_t s);
// Element solves on the matrix cores (every class n <= 32; fdm_mf_ok with
// coarse: the two passes also fit shared memory): mode 0 out = A~^-1 in;
// mode 1 the coarse pass (x_R into cmX, K_e x_R into cmA; in read with the
// coarse rows zeroed and C_1^T nu subtracted when nu is given); mode 2 the full
// solve with the Woodbury correction from cmX and the coarse solution w (with
// kx: from K_e x_R given in kx, [ncm][R], instead of the first pass's x_R).  rc:
// right-hand sides per block (0: the handle's choice).  xslot (mode 1): the
// dual-slot values of the first pass's A~^-1 y as well ([nslots][R]).
bool fdm_mf_ok(const Handle& h, bool coarse);
int fdm_mf_rc(const Handle& h, int R);
void launch_fdm_mf(const Handle& h, int mode, const double2* in, double2* out, int R, hipStream_t s,
                   const double2* nu, const double2* w, int rc = 0, const double2* kx = nullptr,
                   double2* xslot = nullptr);
void launch_extract_kc(const Handle& h, const double2* X, double2* GL, int R, hipStream_t s);
void launch_correct(const Handle& h, double2* X, const double2* w, int R, hipStream_t s);
void launch_gll(const Handle& h, const double2* X, double2* field, int R, int64_t rhs_stride,
                int nrhs_out, hipStream_t s);

// Krylov vector kernels (R must divide 256)
void launch_dots(const double2* V, int64_t vstride, int nvec, const double2* w, int n, int R,
                 double2* part, int nblk, hipStream_t s);
void launch_dots_final(const double2* part, int nblk, int nvec, int R, double2* h, double2* hsum,
                       hipStream_t s);
void launch_update(const double2* V, int64_t vstride, int nvec, const double2* hcoef, double2* w,
                   int n, int R, double sign, hipStream_t s);
void launch_norm(const double2* w, int n, int R, double* part, int nblk, double* nrm, hipStream_t s);
void launch_scale(const double2* w, const double* nrm, double2* out, int n, int R, hipStream_t s);
void launch_axpby(const double2* x, const double2* y, double2* z, int64_t count, double a, double b,
                  hipStream_t s);
void launch_cast_f(const double2* x, float2* y, int64_t count, hipStream_t s);
void launch_cast_d(const float2* x, double2* y, int64_t count, hipStream_t s);
// Nested-dissection coarse solve (device views of the node tables and the factor).
// F (n_K rows) and A (update rows) start at zero and collect the children's
// updates; push[u] < 0 sends update row u to F row -1 - push[u], else to A row push[u].
struct NDView {
  const int* off = nullptr;
  const int64_t* boff = nullptr;
  const int* bnd = nullptr;
  const int64_t* uoff = nullptr;
  const int* push = nullptr;
  const int64_t *mD = nullptr, *mL = nullptr, *mLt = nullptr;
  const double2* fac = nullptr;
  // several columns: two child slots per front row at column stride ld (rows
  // [0, nK) interior, then the update rows; srows = nK + update rows), written by
  // plain stores at push2[u] and zero wherever no child writes
  const int* push2 = nullptr;
  const int* child = nullptr;
  double2* slot = nullptr;
  int64_t ld = 0, srows = 0;
  int nK = 0;
};
// one column: tasks {node, row}; forward U = A - L (g + F)_I pushed to the parent,
// backward X_I = Dinv (g + F)_I - Lt X_B
void launch_nd_fwd1(const ND1Fwd* task, int ntask, const NDView& v, const double2* g, double2* F, double2* A,
                    hipStream_t s);
void launch_nd_bwd1(const ND1Bwd* task, int ntask, const NDView& v, const double2* g, const double2* F, double2* X,
                    hipStream_t s);
// several columns (R <= ld): ntiles output tiles of 32 rows, each split into S
// tasks {node, first row, i0, i1} over the summation; with S > 1 the partial
// tiles go to P (ntiles * S * 32 * 64 values) and a second kernel adds them
void launch_nd_tiles(bool bwd, const int4* task, int ntiles, int S, const NDView& v, const double2* g, double2* X,
                     int R, double2* P, hipStream_t s);
// the top depths as one dense block (several columns): gather the top unknowns'
// right-hand side (g plus the listed front rows' two child slots), scatter the
// block's solution back, and at set-up collect columns of K^-1 restricted to them
void launch_nd_top_gather(int n, const int* idx, const int64_t* gptr, const int* grow, const double2* g,
                          const double2* slot, int64_t ld, int64_t sst, double2* r, int R, hipStream_t s);
void launch_nd_top_scatter(int n, const int* idx, const double2* x, double2* w, int R, hipStream_t s);
void launch_nd_top_collect(int n, const int* idx, const double2* w, int R, int k0, int cols, double2* M,
                           hipStream_t s);
// r = g - K x, K in CSR by row (ptr[n + 1], col, val), [n][R] vectors
void launch_csr_residual(int n, const int64_t* ptr, const int* col, const double2* val, const double2* x,
                         const double2* g, double2* r, int R, hipStream_t s);
void launch_dense_scatter(const int64_t* idx, const double2* val, int64_t nnz, double2* M,
                          hipStream_t s);

void launch_block_scatter(const int* elems, const int64_t* src_off, int nblk, const int64_t* dof_off,
                          const double2* src, double2* full, int R, hipStream_t s);
void launch_fill_zero(double2* x, int64_t count, hipStream_t s);
// per element dJ/d eps_e of J = |E|^2 from the forward field U and the adjoint Lam (one column each)
void launch_eps_gradient(const Handle& h, const double2* U, const double2* Lam, double2 E, double incidence,
                         double* grad, hipStream_t s);
// plane-wave loads (kind 0 total field, 2 scattered field) of the listed elements into columns
// 0..nrhs-1 of B ([dof][R]); the other columns and the other elements are left untouched
void launch_plane_wave_loads(const Handle& h, int kind, const int* elems, int nel, const double* angles, double2* B,
                             int nrhs, int R, hipStream_t s);
// far field of the recovered fields X ([dof][R]) into E ([nrhs_out][nfar]) using h.far
void launch_far_field(const Handle& h, const double2* X, int R, int nrhs_out, double2* E, hipStream_t s);
int dots_blocks(int n, int R);

// Device-resident GMRES (R divides 64; j read from device memory when jptr != nullptr)
struct GmresDims {
  int nchunks = 1, chunk = 1, ngroups = 1, nnorm = 1, step = 1, grid = 1;
  bool wave = false;   // wave-per-item multi-dot (few right-hand sides)
};
// symmetric tiled coarse apply (one right-hand side): tile edge, packing of
// the upper tiles from the dense inverse
int sym_tile_size();
void launch_pack_sym_tiles(const Handle& h, hipStream_t s);
// w = K^-1 g in two steps: per-tile partial products, then their sum per row
void launch_coarse_symv_tiles(const Handle& h, const double2* g, hipStream_t s);
void launch_coarse_symv_reduce(const Handle& h, double2* w, hipStream_t s);
GmresDims gmres_dims(int n, int R, int maxvec);
void launch_mupdate(const double2* V, int64_t vs, const int* jptr, int jfix, const double2* hc, double2* w, int n,
                    int R, double sign, double* npart, hipStream_t s);
void launch_normalize(const double2* w, int n, int R, const GmresDims& g, double* part, double* nrm, double2* out,
                      const int* jptr, int64_t vs, double2* out2, hipStream_t s);
// Arnoldi with delayed reorthogonalisation: multi-dot of the basis, the
// tentative vector V_j and z (2j + 3 entries per chunk, stride dstride), its
// reduction into D, the scalar step (Hessenberg column j-1, Givens, update
// coefficients, j += 1) and the update forming q_j and the next tentative
// vector (also copied to out2)
void launch_dmdot(const double2* V, int64_t vs, const int* jptr, const double2* z, int n, int R, const GmresDims& g,
                  int dstride, double2* part, hipStream_t s);
void launch_dmdot_reduce(const double2* part, const GmresDims& g, const int* jptr, int dstride, int R, double2* D,
                         hipStream_t s);
void launch_dcgs_scalar(int* jptr, const double2* D, double2* Hraw, const double2* hprev, double* rho, double2* uc,
                        double2* H, double2* cs, double2* sn, double2* g, const double* beta, int* done, int* iters,
                        double* resid, double tol, int maxvec, int R, int* counter, int* status, double* hist,
                        hipStream_t s);
void launch_dupdate(double2* V, int64_t vs, const int* jptr, const double2* uc, double2* z, int n, int R,
                    double2* out2, const double2* Hraw, double2* hprev, int maxvec, hipStream_t s);
void launch_gmres_init(const double* nrm, double* beta, double2* g, int* done, int* iters, double* resid, int* jptr,
                       int* counter, int* status, int R, double* hist, hipStream_t s);

}  // namespace hdp
