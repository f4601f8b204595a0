// Internal state of a solver handle and the kernel launch interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hdp.h"
#include "dense.hpp"

namespace hdp {

struct Error {
  hdp_status status;
  std::string msg;
};
[[noreturn]] void fail(hdp_status s, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define HIPCHECK(x) ::hdp::check_hip((x), #x)

// One element class: every element with the same degree, size, material and
// boundary pattern shares all operators below (vertex basis of
// eq. interpolatory_relation, flat mode index ix + n*iy).
struct ElemClass {
  int p = 0, n = 0;
  double hx = 0, hy = 0, eps = 1;
  int bmask = 0;               // bit (s-1): side s on the outer impedance boundary
  int rmask = 0;               // bits 2(s-1)..: Robin-modified side s, 1 gamma = -ik, 2 gamma = +ik
  double sigx = 0, sigy = 0;   // layer stretching s = 1 + i sigma / k per axis
  int top[4] = {1, 1, 1, 1};   // per side: bubbles 2..top are coarse modes
  int gtop[4] = {0, 0, 0, 0};  // per side: bubbles top+1..gtop are dual slots
  int m = 0, nr = 0;           // dual slots, coarse modes
  std::vector<int> R;          // coarse (removed, type-2) modes, canonical order
  std::vector<int> Gam;        // dual-touched type-1 edge modes, slot order
  MatC Ex, Ey;                 // generalised eigenvectors, E^T M~ E = I
  std::vector<cd> Dg;          // (hy/2) lx_i + (hx/2) ly_j, index i + n j
  MatC G;                      // A~^-1 E_R           (n^2 x nr)
  MatC Kc;                     // (E_R^T A~^-1 E_R)^-1 (nr x nr)
  MatC Op1;                    // [D_c ; Phi_c^T]      ((m+nr) x m)
  MatC Phi;                    // Phi_c = -A_11^-1 A_1R = G_Gam Kc on the slots (m x nr)
  MatC Se;                     // Laplace-only Schur complement on Gam (m x m)
  MatC KL;                     // Laplace-only element coarse matrix on R (nr x nr)
  double margin = 0;           // min|Dg| / max|Dg|
  std::vector<int> elems;      // members, leaf indices
};

// Device copies of one precision of the class operators.
template <class T>
struct DevOps {
  T* op1 = nullptr;   // per class, column-major (m+nr) x m
  T* phi = nullptr;   // per class, column-major m x nr
  T* se = nullptr;    // per class, column-major m x m (real part only used)
};

enum KernelFamily {
  KF_SLOT_F = 0, KF_SLOT_P, KF_ASSEMBLE, KF_COARSE, KF_SLOT_COARSE, KF_ROWGATHER, KF_DOTS, KF_UPDATE,
  KF_NORM_SCALE, KF_FDM, KF_ELEMENT_MISC, KF_GLL, KF_CAST, KF_GIVENS, KF_FAR, KF_HBLOCK, KF_COARSE_RED, KF_COUNT
};
extern const char* const KF_NAMES[KF_COUNT];

struct Prof {
  bool on = false;
  bool suspended = false;   // set while an allocation-free call runs (no events created)
  struct Pending { int fam; hipEvent_t a, b; double bytes, flops; };
  std::vector<Pending> pend;
  std::vector<hipEvent_t> pool;
  double ms[KF_COUNT] = {0}, bytes[KF_COUNT] = {0}, flops[KF_COUNT] = {0};
  int64_t n[KF_COUNT] = {0};
};

// One depth of the nested-dissection tree: ranges in the assembly-entry and
// task arrays (R = 1 tasks are rows, other tasks 32-row tiles).
struct NDLevel {
  int f1 = 0, nf1 = 0, b1 = 0, nb1 = 0;
  int fR = 0, nfR = 0, Sf = 1, bR = 0, nbR = 0, Sb = 1;   // first task, tiles, splits per tile
};

// One-column sweep tasks with the node tables already looked up, so that a
// wave starts from one record: forward (row b of node t's L and where its
// update goes) and backward (row i of node t's D^-1 and L^T).
struct ND1Fwd {
  int64_t lrow;   // offset of L_t row b in the factor
  int64_t u;      // update row of (t, b)
  int o, nI;      // node's first unknown and count
  int push, pad;  // destination of the update (as NDHost::push)
};
struct ND1Bwd {
  int64_t drow, lrow;   // offsets of D^-1_t row i and L^T_t row i in the factor
  int64_t bo;           // node's boundary list offset
  int o, nI, nB, i;     // first unknown, count, boundary count, the row
};

// GMRES on the device: iterations queued beyond the one whose status the host
// reads (one keeps the GPU busy on the point source; two measured no faster and
// cost one more iteration past convergence), and status slots in mapped host
// memory (iteration j writes slot j mod STATUS_SLOTS; more slots than
// iterations in flight).  Where one iteration streams long vectors (n_lambda R
// at least GMRES_LONG entries, iterations of a millisecond at 64 columns) the
// host's wait between iterations is small beside the queued iteration that
// would run past convergence, so none is queued.
constexpr int GMRES_AHEAD = 1;
constexpr int64_t GMRES_LONG = int64_t(1) << 20;
constexpr int STATUS_SLOTS = 4;

// Per-block record of the slot kernels (blocks follow the class-grouped element
// order): the element, its class, slot and coarse-mode offsets and counts, and
// the class's operator offsets, so that a block starts with one load.
struct SlotBlock {
  int64_t op1, se, phi;
  int e, c, so, cmo, m, nr, pad0, pad1;
};
// Per-element record of the matrix-core element solves, read with one load.
struct FdmRec {
  int64_t base, eoff, doff, kc;   // element's first coefficient; class's E, 1/D and K_e offsets
  int n, nr, roff, cmo;           // modes per direction, coarse modes, coarse-mode list offset, first coarse mode
  int s0, s1, real, cls;          // dual slots [s0, s1); 1 for a real eigenbasis; the class
};
// Per-slot input gather of the slot kernels: value = a0 v[s0] + a1 v[s1] (an
// index < 0 contributes nothing), the row scalings already multiplied in.
struct SlotIn {
  double a0, a1;
  int s0, s1;
};
// Per-slot output scatter of the preconditioner fused with the row gather: the
// slot's value times coef is added to dual row `row` (each row has at most two
// slots, so two additions onto zero give the same sum in either order).
struct SlotOut {
  double coef;
  int row, pad;
};

struct Handle {
  // problem
  int E = 0, l = 0, nlam = 0, nK = 0;
  int64_t dof = 0;
  double k = 0, discard_tol = 0;
  int max_rhs = 1, max_iter = 100, precision = HDP_FP64;
  double tol = 1e-8;
  int device = 0;                      // the device current at set-up
  hipStream_t stream = nullptr;        // internal stream all work is issued on
  hipStream_t user_stream = nullptr;   // caller's stream; work is ordered after it
  hipEvent_t order_ev = nullptr;
  std::vector<int> deg;
  std::vector<double> eps;
  std::vector<double> ox, oy, hx, hy;   // element origin and size
  std::vector<int> cls;                 // class of each element
  std::vector<ElemClass> classes;
  std::vector<int> bmask;
  std::vector<int> rmask;          // per element, as ElemClass::rmask (zero unless Robin-modified)
  std::vector<double> sigx, sigy;  // per element layer stretching (zero outside layers)
  bool pml = false;
  // per side (4 per element, index 4e + s - 1): 0 outer boundary, 1 conforming,
  // 2 fine side of a hanging edge (one coarser neighbour), 3 coarse side of a
  // hanging edge (several finer neighbours)
  std::vector<int> side_type, side_le;   // side_le: primal rows 0..le on the edge
  std::vector<int> nb_e, nb_s;           // the neighbour (types 1 and 2), -1 otherwise
  std::vector<double> side_a, side_b;    // type 2: s -> t = a s + b into the neighbour's side
  std::vector<std::vector<int>> side_nbrs;   // type 3: the finer neighbours (element indices)
  bool nonconforming = false;
  // offsets
  std::vector<int64_t> dof_off;   // per element, n_e^2 blocks
  std::vector<int> slot_off;      // per element, dual slots
  std::vector<int> cm_off;        // per element, coarse modes
  int nslots = 0, ncm = 0;
  // dual rows: up to two (slot, coef) entries each
  std::vector<int> row_slot;      // 2 * nlam, -1 if absent
  std::vector<double> row_coef;   // 2 * nlam
  std::vector<double> row_xinv;   // 1 / (C_1 C_1^T)_rr
  std::vector<int> slot_row;      // per slot
  std::vector<double> slot_coef;
  std::vector<int> slot_mode;     // per slot, local mode index (for full arrays)
  // coarse map: each coarse mode i (element-local removed mode) is a linear
  // combination T of global coarse unknowns (a single unit entry except on
  // the fine side of a hanging edge and at hanging points)
  std::vector<int> t_ptr, t_dof;         // CSR over coarse modes
  std::vector<double> t_coef;
  std::vector<int> cdof_ptr, cdof_list;  // transpose: coarse unknown -> coarse modes
  std::vector<double> cdof_coef;
  std::vector<int> cm_mode;       // per coarse mode, local mode index
  std::vector<double> dof_x, dof_y;   // per coarse unknown: position of its vertex or edge midpoint
  std::vector<char> dof_vtx;          // per coarse unknown: 1 for a mesh vertex
  // coarse factor: 0 dense inverse of K (coarse unknowns in breadth-first level
  // order), 2 nested-dissection multifrontal factor: tree nodes in postorder, node t
  // owns the coarse unknowns [nd_off[t], nd_off[t+1]) and, after its subtree is
  // eliminated, couples to the ancestor unknowns nd_bnd[nd_boff[t] .. nd_boff[t+1])
  int coarse_mode = -1;            // -1: chosen by size at setup
  std::vector<int> nd_off, nd_depth, nd_child;
  std::vector<int64_t> nd_boff;
  std::vector<int> nd_bnd;
  std::vector<NDLevel> nd_levels;   // per tree depth
  int nd_split = 1024;              // workgroups a depth's split tiles aim at (several columns)
  int dn_ntiles = 0, dn_S = 1;      // dense inverse at several columns: output tiles, splits
  int64_t nd_P_tasks = 0;           // partial tiles nd_P holds
  size_t nd_tR_cap[2] = {0, 0};     // capacity of nd_tRf / nd_tRb
  bool coarse_refine = false;       // refine each coarse solve once (set at setup from the check)
  int cmA_b_R = 0;                  // columns of d.cmA_b valid for the current loads (0: none)
  // nested dissection at several columns: the depths above nd_top_depth solved as
  // one dense block (the top unknowns' rows of K^-1), nd_top_n unknowns (0: off)
  int nd_top_depth = 0, nd_top_n = 0, nd_top_ntiles = 0, nd_top_S = 1;
  std::vector<int> nd_top_host;     // the top unknowns (nested-dissection indices)
  double nd_top_check = 0;          // set-up check of the block: ||K x - b|| / ||b||
  double coarse_check = 0;         // relative residual of the coarse factor on a test vector
  int sym_nt = 0, sym_ntiles = 0;   // tile rows and upper tiles of the symmetric coarse inverse
  double coarse_bytes1 = 0;         // factor bytes of a one-RHS coarse solve (half with the tiles)
  double coarse_bytes = 0, coarse_flops = 0;   // per coarse solve and RHS column (flops), factor bytes
  double coarse_band_bytes = 0;   // a banded (envelope) LU factor of K in natural order, bytes
  // C_2 (dual rows x coarse unknowns), non-zero only on hanging edges
  std::vector<int> c2_ptr, c2_dof, c2t_ptr, c2t_row;
  std::vector<double> c2_coef, c2t_coef;
  // preconditioner blocks on the dual rows that C_2 couples (hanging edges):
  // per block the rows, X^-1 and Y_2, dense column-major
  std::vector<int> hb_off, hb_rows;
  std::vector<int64_t> hb_moff;
  std::vector<double> hb_xinv, hb_y2;
  int nh = 0;
  // class-sorted element order and launch tables
  std::vector<int> order;         // elements grouped by class
  // per degree n: Gauss-Legendre rule with n+40 nodes and the vertex basis there
  std::map<int, std::vector<double>> quad_x, quad_w, quad_N;
  double min_margin = 1;
  double setup_ms = 0;
  double setup_host_ms = 0, setup_classes_ms = 0, setup_coarse_ms = 0;   // set-up phases (host analysis in total,
                                                                         // its class operators, the coarse factor)
  // algorithmic work per right-hand side (bytes of class operators are
  // counted once per launch, like any operand read from memory once)
  double op1_bytes = 0, se_bytes = 0, phi_bytes = 0;
  double flops_F = 0, flops_P = 0, flops_coarse = 0, flops_fdm = 0, flops_gll = 0, flops_fdm_coarse = 0;

  // device buffers --------------------------------------------------------
  struct Dev {
    // maps
    int *elem_cls = nullptr, *order = nullptr, *slot_off = nullptr, *cm_off = nullptr;
    SlotBlock* slot_blk = nullptr;
    SlotIn* slot_in[3] = {nullptr, nullptr, nullptr};   // modes 0 (F), 1 (P, rows), 2 (P, slots)
    SlotOut* slot_out = nullptr;
    int64_t* dof_off = nullptr;
    int *row_slot = nullptr, *slot_row = nullptr, *slot_mode = nullptr;
    int64_t *slot_pos = nullptr, *cm_pos = nullptr;   // positions in full-element arrays
    double *row_coef = nullptr, *row_xinv = nullptr, *slot_coef = nullptr;
    int *t_ptr = nullptr, *t_dof = nullptr, *cdof_ptr = nullptr, *cdof_list = nullptr, *cm_mode = nullptr;
    double *t_coef = nullptr, *cdof_coef = nullptr;
    // the identity expansion with coefficient -1 (coarse mode i -> entry i of a
    // [ncm][R] array): the slot coarse correction then applies -Phi to
    // per-element coarse values instead of Phi T_e w
    int *id_ptr = nullptr, *id_dof = nullptr;
    double* id_coef = nullptr;
    int *c2_ptr = nullptr, *c2_dof = nullptr, *c2t_ptr = nullptr, *c2t_row = nullptr;
    double *c2_coef = nullptr, *c2t_coef = nullptr;
    int *hb_off = nullptr, *hb_rows = nullptr, *hb_blk = nullptr;
    int64_t* hb_moff = nullptr;
    double *hb_xinv = nullptr, *hb_y2 = nullptr;
    double2 *hb_tmp = nullptr, *fv = nullptr, *pv = nullptr;
    double2 *adj_u = nullptr, *adj_g = nullptr, *adj_E = nullptr;   // adjoint gradient work
    double* adj_grad = nullptr;
    double* cls_M = nullptr;   // per class the 1-D vertex mass matrix (n x n)
    int64_t* cls_Moff = nullptr;
    // nested-dissection coarse factor
    double2 *nd_fac = nullptr, *nd_FA = nullptr;   // FA: front accumulators, n_K then update rows
    int *nd_off = nullptr, *nd_bnd = nullptr, *nd_push = nullptr;
    int64_t *nd_boff = nullptr, *nd_uoff = nullptr, *nd_mD = nullptr, *nd_mL = nullptr, *nd_mLt = nullptr;
    int64_t nd_urows = 0;
    ND1Fwd* nd_f1 = nullptr;
    ND1Bwd* nd_b1 = nullptr;
    // one step of iterative refinement of the coarse solve (when the factor alone
    // misses 1e-10): K in CSR by row, residual and correction buffers
    int64_t* k_ptr = nullptr;
    int* k_col = nullptr;
    double2 *k_val = nullptr, *nd_r = nullptr, *nd_dx = nullptr;
    int4 *nd_tRf = nullptr, *nd_tRb = nullptr;
    double2* nd_P = nullptr;   // partial tiles of the split top levels
    double2* nd_slot = nullptr;   // two child slots per front row, [2][nK + urows][Rp], zero from set-up
    // dense inverse at several columns through the tile kernels (a one-node tree)
    int4* dn_tasks = nullptr;
    int *dn_off = nullptr, *dn_int = nullptr;   // dn_int: children {-1, -1}, then a zero
    int64_t *dn_boff = nullptr, *dn_zero64 = nullptr;
    double2* dn_P = nullptr;
    int *nd_push2 = nullptr, *nd_childv = nullptr;
    // the dense top block (several columns): its unknowns, their gather lists of
    // front rows, the block (row-major), work arrays [n][R_max] and tile tasks
    int *nd_top_idx = nullptr, *nd_top_grow = nullptr, *nd_top_off = nullptr, *nd_top_int = nullptr;
    int64_t *nd_top_gptr = nullptr, *nd_top_boff = nullptr, *nd_top_zero64 = nullptr;
    double2 *nd_top_inv = nullptr, *nd_top_r = nullptr, *nd_top_x = nullptr, *nd_top_P = nullptr;
    int4* nd_top_tasks = nullptr;
    int64_t nd_ld = 0;
    // per-class tables
    int *cls_n = nullptr, *cls_m = nullptr, *cls_nr = nullptr;
    int* cls_real = nullptr;   // 1 when the class's eigenbasis is real
    FdmRec* fdm_rec = nullptr; // per element
    int64_t *cls_op1 = nullptr, *cls_phi = nullptr, *cls_se = nullptr;   // offsets
    int64_t *cls_E = nullptr, *cls_D = nullptr, *cls_G = nullptr, *cls_Kc = nullptr, *cls_V = nullptr;
    int* cls_gam = nullptr;   // per class offset into gam_modes
    int* gam_modes = nullptr;
    int* cls_R = nullptr;     // per class offset into r_modes
    int* r_modes = nullptr;
    // operators
    double2 *op1 = nullptr, *phi = nullptr;   // FP64
    double2* se = nullptr;
    float2 *op1_f = nullptr, *phi_f = nullptr; // FP32 copies
    float2* se_f = nullptr;
    double2* mass_fac = nullptr;   // per element s_x s_y (layers only; null without layers)
    double2 *Ex = nullptr, *Ey = nullptr, *Dinv = nullptr, *G = nullptr, *Kc = nullptr;
    double* V = nullptr;      // GLL sampling matrices per class
    double2* Kinv = nullptr;  // nK x nK (symmetric)
    // the same inverse as its upper 64 x 64 tiles (one-RHS coarse apply)
    double2 *Ksym = nullptr, *sym_part = nullptr;
    int2* sym_tij = nullptr;
    // work
    double2 *slotA = nullptr, *slotB = nullptr, *cmA = nullptr, *gK = nullptr, *wK = nullptr;
    double2* cmX = nullptr;   // [ncm][R]: coarse-mode values x_R of the element solve's first pass
    double2* cmA_b = nullptr; // [ncm][R]: K_e x_R of the loads alone (the interface right-hand side's pass)
    float2 *slotA_f = nullptr, *slotB_f = nullptr, *cmA_f = nullptr;
    double2 *full0 = nullptr, *full1 = nullptr;   // [dof][R]
    double2 *V_kry = nullptr;                      // (max_iter+1) x nlam x R
    double2 *w = nullptr, *t0 = nullptr, *t1 = nullptr, *t2 = nullptr;
    double2* part = nullptr;
    // Arnoldi with delayed reorthogonalisation: reduced dots, unrotated
    // Hessenberg columns, first-pass coefficients, update coefficients, scale
    // of the tentative vector
    double2 *dots = nullptr, *Hraw = nullptr, *hprev = nullptr, *ucoef = nullptr;
    double* rho = nullptr;
    double *nrm = nullptr, *npart = nullptr;
    float2* vf = nullptr;
    double2 *vcur = nullptr, *Hdev = nullptr, *cs = nullptr, *sn = nullptr, *gvec = nullptr;
    double *beta = nullptr, *resid = nullptr, *hist = nullptr;   // hist: (max_iter+1) x R
    int *jdev = nullptr, *counter = nullptr, *status = nullptr, *done = nullptr, *iters = nullptr;
    int* status_host = nullptr;   // pinned, mapped, coherent: STATUS_SLOTS pairs of ints
    int* status_hdev = nullptr;   // the same memory as the device addresses it
    int* load_elems = nullptr;
    int64_t* load_off = nullptr;
    double2* load_vals = nullptr;
    // plane-wave load tables: per class the Gauss rule (q nodes) and the vertex basis there
    int *cls_q = nullptr, *bmask = nullptr, *pw_elems = nullptr;
    int64_t* cls_qoff = nullptr;
    double *qx = nullptr, *qw = nullptr, *qN = nullptr, *ox = nullptr, *oy = nullptr, *hx = nullptr, *hy = nullptr,
           *eps = nullptr, *angles = nullptr;
    int n_pw_elems = 0, pw_kind = -1;
    double2* ycoef = nullptr;
  } d;
  std::vector<void*> allocations;
  hdp_allocator allocator{};   // the caller's device-memory pair, or zero for hipMalloc / hipFree
  Prof prof;
  // far-field geometry of the last request (device arrays, grown on demand)
  struct Far {
    int nsides = 0, nq = 0, nfar = 0;
    std::vector<uint8_t> inside;
    std::vector<double> angles;
    int *elem = nullptr, *side = nullptr, *node_off = nullptr;
    int64_t* tab_off = nullptr;
    double *tab = nullptr, *dscale = nullptr, *px = nullptr, *py = nullptr, *pw = nullptr, *pnx = nullptr,
           *pny = nullptr, *ang = nullptr;
    double2 *U = nullptr, *DU = nullptr;
    int capR = 0;
  } far;
  void* rocblas = nullptr;   // rocblas_handle for the batched coarse solve
  bool use_graphs = false;
  int fdm_rc = 0;    // right-hand sides per block of the matrix-core element solve (0: heuristic)
  int slot_rb = 32;  // right-hand sides per block of the matrix-core slot operators (16, 32, 64)
  struct Tune {
    std::string kernel;
    int cols;
    double ms;
    bool chosen;
  };
  std::vector<Tune> tune;   // the set-up autotuner's measurements
  std::vector<double> last_hist;   // residual history of the last GMRES run, [iteration][R]
  int last_hist_R = 0, last_hist_len = 0;
  double t_launch = 0, t_wait = 0;
  size_t load_cap_blocks = 0, load_cap_vals = 0;   // host time in GMRES launch calls / waits (ms)
  std::map<std::tuple<int, int, double>, hipGraphExec_t> graphs;   // (R, precision, tol)
};

// Brackets the launches issued during its lifetime with profiling events.
struct Timed {
  Handle& h;
  int fam;
  double bytes, flops;
  hipEvent_t a = nullptr;
  Timed(Handle& h_, int fam_, double bytes_, double flops_);
  ~Timed();
};
void prof_flush(Handle& h);   // after a stream synchronisation

// Work buffers of the preconditioner application (P^-1 v at R columns): slot
// values in FP64 or FP32, the FP32 copy of v, and on meshes with hanging edges
// X^-1 v and the hanging-block intermediate.
struct PWork {
  double2* slot;     // [nslots][R]
  float2* slot_f;    // [nslots][R] (mixed precision)
  float2* vf;        // [nlam][R]   (mixed precision)
  double2* pv;       // [nlam][R]   (hanging edges)
  double2* hb_tmp;   // [nh][R]     (hanging edges)
};
void apply_P_ws(Handle& h, const double2* v, double2* u, int R, int prec, const PWork& w);

// noalloc.hip: the device-resident scratch array of the allocation-free entry
// point.  scratch_init resolves its address on the current device (once per
// device; called at set-up); scratch_ptr returns it for a device (null if not
// resolved); SCRATCH_BYTES is its size.
extern const size_t SCRATCH_BYTES;
void scratch_init(int device);
void* scratch_ptr(int device);

// setup.cpp
void build_host(Handle& h, const hdp_mesh* mesh, const hdp_problem* prob);
// Coarse matrix K = sum_e T_e^T Kc_e T_e as sorted COO (key = row + nK * col).
void coarse_coo(const Handle& h, std::vector<int64_t>& kidx, std::vector<double2>& kval);
double coarse_band_bytes(int nK, const std::vector<int64_t>& kidx);

// coarse_nd.cpp: the nested-dissection factor assembled on the host.  Per node
// the blocks Dinv (nI x nI), L (nB x nI) and Lt = L^T, row-major, back to back in
// fac; update rows (uoff) hold the boundary entries of the nodes' fronts, and
// push names each row's place in the parent's front (-1 - unknown for a row the
// parent owns, else the parent's update row).  Per tree depth: the row tasks of
// the device sweeps.
struct NDHost {
  std::vector<double2> fac;
  std::vector<int64_t> uoff, mD, mL, mLt;
  int64_t urows = 0;
  std::vector<int> push;
  std::vector<int> push2;     // slot row of each update row (several columns)
  std::vector<int2> t1f, t1b;
  std::vector<int4> tRf, tRb;
  std::vector<NDLevel> levels;
  int64_t part_tasks = 0;     // largest split level (tiles x splits)
  double flops_per_col = 0;   // 8 (nI^2 + 2 nB nI) summed over the nodes
};
void nd_factor(const Handle& h, const std::vector<int64_t>& kidx, const std::vector<double2>& kval, NDHost& f);
// every device block of the handle back through its allocator (or hipFree)
void release_allocations(Handle& h);
// the row tasks alone (levels, t1f/t1b, tRf/tRb, part_tasks) for a split target;
// ND_SPLITS are the targets the set-up autotuner tries
void nd_tasks(const Handle& h, NDHost& f, int target);
constexpr int ND_SPLITS[] = {256, 512, 1024, 2048};
// most unknowns of the dense top block of the nested-dissection sweeps
constexpr int64_t ND_TOP_MAX = 3072;
void build_device(Handle& h);
// Element loads of the elements with a non-zero load: elems lists them and
// vals holds their blocks back to back, each [n_e^2][R].
void compute_loads(const Handle& h, const hdp_rhs* rhs, int R, std::vector<int>& elems, std::vector<cd>& vals);

}  // namespace hdp
