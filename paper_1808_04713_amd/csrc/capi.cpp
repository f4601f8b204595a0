// C ABI of the solver: device setup, operator entry points and the GMRES
// driver (paper Sec. 2.3.1 and 2.3.4; GMRES-IR for the mixed-precision path).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "basis.hpp"
#include "internal.hpp"
#include "kernels.hpp"

struct hdp_handle {
  hdp::Handle h;
};

namespace hdp {

namespace {
thread_local std::string g_err;

int pow2ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

template <class T>
T* dalloc(Handle& h, size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    fail(HDP_E_NOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  h.allocations.push_back(p);
  return static_cast<T*>(p);
}

template <class T>
T* upload(Handle& h, const std::vector<T>& v) {
  T* p = dalloc<T>(h, v.size());
  if (!v.empty()) HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

std::vector<double2> pack_c(const std::vector<cd>& v) {
  std::vector<double2> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = make_double2(v[i].real(), v[i].imag());
  return o;
}

}  // namespace

[[noreturn]] void fail(hdp_status s, const std::string& msg) { throw Error{s, msg}; }

const char* const KF_NAMES[KF_COUNT] = {"slot_apply_F", "slot_apply_P", "coarse_assemble", "coarse_gemv",
                                        "slot_coarse", "row_gather", "gmres_dots", "gmres_update",
                                        "gmres_norm_scale", "fdm_local_solve", "element_coarse_fix",
                                        "gll_sample", "precision_cast"};

static hipEvent_t prof_event(Handle& h) {
  if (!h.prof.pool.empty()) {
    hipEvent_t e = h.prof.pool.back();
    h.prof.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHECK(hipEventCreate(&e));
  return e;
}

Timed::Timed(Handle& h_, int fam_, double bytes_, double flops_) : h(h_), fam(fam_), bytes(bytes_), flops(flops_) {
  if (!h.prof.on) return;
  a = prof_event(h);
  HIPCHECK(hipEventRecord(a, h.stream));
}

Timed::~Timed() {
  if (!h.prof.on || !a) return;
  hipEvent_t b = prof_event(h);
  if (hipEventRecord(b, h.stream) != hipSuccess) return;
  h.prof.pend.push_back({fam, a, b, bytes, flops});
}

void prof_flush(Handle& h) {
  for (auto& p : h.prof.pend) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      h.prof.ms[p.fam] += ms;
      h.prof.n[p.fam] += 1;
      h.prof.bytes[p.fam] += p.bytes;
      h.prof.flops[p.fam] += p.flops;
    }
    h.prof.pool.push_back(p.a);
    h.prof.pool.push_back(p.b);
  }
  h.prof.pend.clear();
}

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(HDP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void build_device(Handle& h) {
  auto& d = h.d;
  int E = h.E;
  d.elem_cls = upload(h, h.cls);
  d.order = upload(h, h.order);
  d.slot_off = upload(h, h.slot_off);
  d.cm_off = upload(h, h.cm_off);
  d.dof_off = upload(h, h.dof_off);
  d.row_slot = upload(h, h.row_slot);
  d.row_coef = upload(h, h.row_coef);
  d.row_xinv = upload(h, h.row_xinv);
  d.slot_row = upload(h, h.slot_row);
  d.slot_coef = upload(h, h.slot_coef);
  d.slot_mode = upload(h, h.slot_mode);
  d.cm_dof = upload(h, h.cm_dof);
  d.cdof_ptr = upload(h, h.cdof_ptr);
  d.cdof_list = upload(h, h.cdof_list);
  d.cm_mode = upload(h, h.cm_mode);
  std::vector<int64_t> slot_pos(h.nslots), cm_pos(h.ncm);
  for (int e = 0; e < E; ++e) {
    for (int s = h.slot_off[e]; s < h.slot_off[e + 1]; ++s) slot_pos[s] = h.dof_off[e] + h.slot_mode[s];
    for (int i = h.cm_off[e]; i < h.cm_off[e + 1]; ++i) cm_pos[i] = h.dof_off[e] + h.cm_mode[i];
  }
  d.slot_pos = upload(h, slot_pos);
  d.cm_pos = upload(h, cm_pos);
  // class tables and operators
  int NC = int(h.classes.size());
  std::vector<int> cn(NC), cm(NC), cnr(NC), cgam(NC), cR(NC);
  std::vector<int64_t> o_op1(NC), o_phi(NC), o_se(NC), o_E(NC), o_D(NC), o_G(NC), o_Kc(NC), o_V(NC);
  std::vector<double2> op1, phi, Ex, Ey, Dinv, G, Kc;
  std::vector<double> se, V;
  std::vector<int> gam, rmod;
  for (int c = 0; c < NC; ++c) {
    const ElemClass& C = h.classes[c];
    cn[c] = C.n; cm[c] = C.m; cnr[c] = C.nr;
    o_op1[c] = op1.size(); o_phi[c] = phi.size(); o_se[c] = se.size();
    o_E[c] = Ex.size(); o_D[c] = Dinv.size(); o_G[c] = G.size(); o_Kc[c] = Kc.size(); o_V[c] = V.size();
    cgam[c] = gam.size(); cR[c] = rmod.size();
    for (auto& v : C.Op1.a) op1.push_back(make_double2(v.real(), v.imag()));
    for (auto& v : C.Phi.a) phi.push_back(make_double2(v.real(), v.imag()));
    for (auto& v : C.Se.a) se.push_back(v);
    for (auto& v : C.Ex.a) Ex.push_back(make_double2(v.real(), v.imag()));
    for (auto& v : C.Ey.a) Ey.push_back(make_double2(v.real(), v.imag()));
    for (auto& v : C.Dg) { cd iv = 1.0 / v; Dinv.push_back(make_double2(iv.real(), iv.imag())); }
    for (auto& v : C.G.a) G.push_back(make_double2(v.real(), v.imag()));
    for (auto& v : C.Kc.a) Kc.push_back(make_double2(v.real(), v.imag()));
    std::vector<double> t = gll_nodes(C.n), row(C.n);
    std::vector<double> Vc(size_t(C.n) * C.n);
    for (int i = 0; i < C.n; ++i) {
      vertex_basis(C.n, t[i], row.data());
      for (int a = 0; a < C.n; ++a) Vc[i + size_t(C.n) * a] = row[a];
    }
    V.insert(V.end(), Vc.begin(), Vc.end());
    gam.insert(gam.end(), C.Gam.begin(), C.Gam.end());
    rmod.insert(rmod.end(), C.R.begin(), C.R.end());
  }
  d.cls_n = upload(h, cn); d.cls_m = upload(h, cm); d.cls_nr = upload(h, cnr);
  d.cls_op1 = upload(h, o_op1); d.cls_phi = upload(h, o_phi); d.cls_se = upload(h, o_se);
  d.cls_E = upload(h, o_E); d.cls_D = upload(h, o_D); d.cls_G = upload(h, o_G);
  d.cls_Kc = upload(h, o_Kc); d.cls_V = upload(h, o_V);
  d.cls_gam = upload(h, cgam); d.gam_modes = upload(h, gam);
  d.cls_R = upload(h, cR); d.r_modes = upload(h, rmod);
  d.op1 = upload(h, op1); d.phi = upload(h, phi); d.se = upload(h, se);
  std::vector<float2> op1f(op1.size()), phif(phi.size());
  std::vector<float> sef(se.size());
  for (size_t i = 0; i < op1.size(); ++i) op1f[i] = make_float2(float(op1[i].x), float(op1[i].y));
  for (size_t i = 0; i < phi.size(); ++i) phif[i] = make_float2(float(phi[i].x), float(phi[i].y));
  for (size_t i = 0; i < se.size(); ++i) sef[i] = float(se[i]);
  d.op1_f = upload(h, op1f); d.phi_f = upload(h, phif); d.se_f = upload(h, sef);
  d.Ex = upload(h, Ex); d.Ey = upload(h, Ey); d.Dinv = upload(h, Dinv);
  d.G = upload(h, G); d.Kc = upload(h, Kc); d.V = upload(h, V);
  // coarse matrix K = sum_e T_e^T Kc T_e (summed on the host, scattered densely)
  std::vector<std::pair<int64_t, cd>> coo;
  for (int e = 0; e < E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    for (int b = 0; b < C.nr; ++b)
      for (int a = 0; a < C.nr; ++a) {
        int64_t i = h.cm_dof[h.cm_off[e] + a], j = h.cm_dof[h.cm_off[e] + b];
        coo.push_back({i + int64_t(h.nK) * j, C.Kc(a, b)});
      }
  }
  std::sort(coo.begin(), coo.end(), [](auto& x, auto& y) { return x.first < y.first; });
  std::vector<int64_t> kidx;
  std::vector<double2> kval;
  for (size_t t = 0; t < coo.size();) {
    int64_t key = coo[t].first;
    cd s = 0;
    while (t < coo.size() && coo[t].first == key) s += coo[t++].second;
    kidx.push_back(key);
    kval.push_back(make_double2(s.real(), s.imag()));
  }
  size_t nK = size_t(h.nK);
  d.Kinv = dalloc<double2>(h, nK * nK);
  HIPCHECK(hipMemsetAsync(d.Kinv, 0, nK * nK * sizeof(double2), h.stream));
  int64_t* didx = upload(h, kidx);
  double2* dval = upload(h, kval);
  launch_dense_scatter(didx, dval, int64_t(kidx.size()), d.Kinv, h.stream);
  rocblas_handle rb;
  if (rocblas_create_handle(&rb) != rocblas_status_success) fail(HDP_E_DEVICE, "rocblas_create_handle");
  rocblas_set_stream(rb, h.stream);
  int* ipiv = dalloc<int>(h, nK);
  int* info = dalloc<int>(h, 1);
  rocblas_status st = rocsolver_zgetrf(rb, h.nK, h.nK, (rocblas_double_complex*)d.Kinv, h.nK, ipiv, info);
  int hinfo = 0;
  if (st == rocblas_status_success) {
    HIPCHECK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, h.stream));
    HIPCHECK(hipStreamSynchronize(h.stream));
  }
  if (st == rocblas_status_success && hinfo == 0)
    st = rocsolver_zgetri(rb, h.nK, (rocblas_double_complex*)d.Kinv, h.nK, ipiv, info);
  if (st == rocblas_status_success && hinfo == 0) {
    HIPCHECK(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, h.stream));
    HIPCHECK(hipStreamSynchronize(h.stream));
  }
  rocblas_destroy_handle(rb);
  if (st != rocblas_status_success) fail(HDP_E_DEVICE, "rocsolver failed on the coarse matrix");
  if (hinfo != 0) fail(HDP_E_COARSE, "coarse matrix K is singular");
  // work buffers sized for the largest RHS batch (padded to a power of two)
  size_t Rp = size_t(pow2ceil(h.max_rhs));
  size_t nl = size_t(h.nlam);
  d.slotA = dalloc<double2>(h, size_t(h.nslots) * Rp);
  d.slotB = dalloc<double2>(h, size_t(h.nslots) * Rp);
  d.slotA_f = dalloc<float2>(h, size_t(h.nslots) * Rp);
  d.slotB_f = dalloc<float2>(h, size_t(h.nslots) * Rp);
  d.cmA = dalloc<double2>(h, size_t(h.ncm) * Rp);
  d.cmA_f = dalloc<float2>(h, size_t(h.ncm) * Rp);
  d.gK = dalloc<double2>(h, nK * Rp);
  d.wK = dalloc<double2>(h, nK * Rp);
  d.full0 = dalloc<double2>(h, size_t(h.dof) * Rp);
  d.full1 = dalloc<double2>(h, size_t(h.dof) * Rp);
  d.V_kry = dalloc<double2>(h, (size_t(h.max_iter) + 1) * nl * Rp);
  d.w = dalloc<double2>(h, nl * Rp);
  d.t0 = dalloc<double2>(h, nl * Rp);
  d.t1 = dalloc<double2>(h, nl * Rp);
  d.t2 = dalloc<double2>(h, nl * Rp);
  d.vf = dalloc<float2>(h, nl * Rp);
  d.hbuf = dalloc<double2>(h, (size_t(h.max_iter) + 1) * Rp);
  d.hsum = dalloc<double2>(h, (size_t(h.max_iter) + 1) * Rp);
  d.part = dalloc<double2>(h, size_t(512) * (h.max_iter + 1) * Rp);
  d.npart = dalloc<double>(h, size_t(512) * Rp);
  d.nrm = dalloc<double>(h, Rp);
  d.ycoef = dalloc<double2>(h, (size_t(h.max_iter) + 1) * Rp);
  HIPCHECK(hipStreamSynchronize(h.stream));
}

// ---------------------------------------------------------------------------
// Operators on dual vectors ([nlam][R]).
void apply_F(Handle& h, const double2* v, double2* u, int R, int prec) {
  auto& d = h.d;
  hipStream_t s = h.stream;
  const double c = 16.0 * R, nsl = h.nslots, ncm = h.ncm, nl = h.nlam, nK = h.nK;
  const double cw = prec == HDP_FP64 ? 16.0 * R : 8.0 * R;   // bytes per value of the local operators
  const double ob = prec == HDP_FP64 ? 1.0 : 0.5;
  if (prec != HDP_FP64) {
    Timed t(h, KF_CAST, nl * (c + cw), 0);
    launch_cast_f(v, d.vf, int64_t(h.nlam) * R, s);
  }
  {
    Timed t(h, KF_SLOT_F, nsl * cw * 2 + ncm * cw + ob * h.op1_bytes, h.flops_F * R);
    if (prec == HDP_FP64) launch_slot_apply<double2>(h, 0, v, d.slotA, d.cmA, R, s);
    else launch_slot_apply<float2>(h, 0, d.vf, d.slotA_f, d.cmA_f, R, s);
  }
  {
    Timed t(h, KF_ASSEMBLE, ncm * cw + nK * c, 0);
    if (prec == HDP_FP64) launch_assemble<double2>(h, d.cmA, nullptr, d.gK, R, s);
    else launch_assemble<float2>(h, d.cmA_f, nullptr, d.gK, R, s);
  }
  {
    Timed t(h, KF_COARSE, nK * nK * 16.0 + 2 * nK * c, 8.0 * nK * nK * R);
    launch_coarse_solve(h, d.gK, d.wK, R, s);
  }
  {
    Timed t(h, KF_SLOT_COARSE, nsl * cw * 2 + ncm * c + ob * h.phi_bytes, h.flops_coarse * R);
    if (prec == HDP_FP64) launch_slot_coarse<double2>(h, d.slotA, d.wK, d.slotB, R, s);
    else launch_slot_coarse<float2>(h, d.slotA_f, d.wK, d.slotB_f, R, s);
  }
  {
    Timed t(h, KF_ROWGATHER, nsl * cw + nl * c, 0);
    if (prec == HDP_FP64) launch_rowgather<double2>(h, d.slotB, false, false, u, R, s);
    else launch_rowgather<float2>(h, d.slotB_f, false, false, u, R, s);
  }
}

void apply_P(Handle& h, const double2* v, double2* u, int R, int prec) {
  auto& d = h.d;
  hipStream_t s = h.stream;
  const double c = 16.0 * R, nsl = h.nslots, nl = h.nlam;
  const double cw = prec == HDP_FP64 ? 16.0 * R : 8.0 * R;
  const double ob = prec == HDP_FP64 ? 1.0 : 0.5;
  if (prec != HDP_FP64) {
    Timed t(h, KF_CAST, nl * (c + cw), 0);
    launch_cast_f(v, d.vf, int64_t(h.nlam) * R, s);
  }
  {
    Timed t(h, KF_SLOT_P, nsl * cw * 2 + ob * h.se_bytes, h.flops_P * R);
    if (prec == HDP_FP64) launch_slot_apply<double2>(h, 1, v, d.slotA, nullptr, R, s);
    else launch_slot_apply<float2>(h, 1, d.vf, d.slotA_f, nullptr, R, s);
  }
  {
    Timed t(h, KF_ROWGATHER, nsl * cw + nl * c, 0);
    if (prec == HDP_FP64) launch_rowgather<double2>(h, d.slotA, false, true, u, R, s);
    else launch_rowgather<float2>(h, d.slotA_f, false, true, u, R, s);
  }
}

// Solve A^ [x_I; x_R] = [y_I; y_R] element-wise (eq. block_matrix_inversion):
// X holds y_I on entry (coarse modes ignored) and the element solution on exit;
// y_R is assembled from Bfull's coarse modes (or zero when Bfull is null).
void element_solve(Handle& h, double2* X, const double2* Bfull, int R) {
  auto& d = h.d;
  hipStream_t s = h.stream;
  const double c = 16.0 * R, dof = double(h.dof), ncm = h.ncm, nK = h.nK;
  {
    Timed t(h, KF_ELEMENT_MISC, ncm * c, 0);
    launch_zero_R(h, X, R, s);
  }
  {
    Timed t(h, KF_FDM, 2 * dof * c, h.flops_fdm * R);
    launch_fdm(h, X, X, R, s);
  }
  {
    Timed t(h, KF_ELEMENT_MISC, 2 * ncm * c, 0);
    launch_extract_kc(h, X, d.cmA, R, s);
  }
  {
    Timed t(h, KF_ASSEMBLE, 2 * ncm * c + nK * c, 0);
    launch_assemble<double2>(h, d.cmA, Bfull, d.gK, R, s);
  }
  {
    Timed t(h, KF_COARSE, nK * nK * 16.0 + 2 * nK * c, 8.0 * nK * nK * R);
    launch_coarse_solve(h, d.gK, d.wK, R, s);
  }
  {
    Timed t(h, KF_ELEMENT_MISC, 2 * dof * c + ncm * c, 0);
    launch_correct(h, X, d.wK, R, s);
  }
}

// Interface right-hand side g = C_1 x_I with x_I from the element loads in full0.
void interface_rhs(Handle& h, double2* g, int R) {
  auto& d = h.d;
  HIPCHECK(hipMemcpyAsync(d.full1, d.full0, size_t(h.dof) * R * sizeof(double2), hipMemcpyDeviceToDevice,
                          h.stream));
  element_solve(h, d.full1, d.full0, R);
  Timed t(h, KF_ROWGATHER, h.nslots * 16.0 * R + h.nlam * 16.0 * R, 0);
  launch_rowgather<double2>(h, d.full1, true, false, g, R, h.stream);
}

struct GmresResult {
  std::vector<int> iters;
  std::vector<double> rel;
};

// Left-preconditioned GMRES with CGS2 on R systems at once (x0 = 0); stops
// each system when ||P^-1 r_k|| / ||P^-1 r_0|| <= tol.  x receives the iterate.
GmresResult gmres(Handle& h, const double2* rhs, double2* x, int R, int prec, double tol, int max_iter) {
  auto& d = h.d;
  hipStream_t s = h.stream;
  int n = h.nlam;
  int64_t vs = int64_t(n) * R;
  int nblk = dots_blocks(n, R);
  GmresResult res;
  res.iters.assign(R, 0);
  res.rel.assign(R, 1.0);
  HIPCHECK(hipMemsetAsync(x, 0, size_t(vs) * sizeof(double2), s));
  // V_0 = P^-1 rhs / beta
  apply_P(h, rhs, d.w, R, prec);
  launch_norm(d.w, n, R, d.npart, nblk, d.nrm, s);
  std::vector<double> beta(R);
  HIPCHECK(hipMemcpyAsync(beta.data(), d.nrm, R * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  launch_scale(d.w, d.nrm, d.V_kry, n, R, s);
  std::vector<std::vector<cd>> H(R), cs(R), sn(R), gv(R);
  std::vector<int> done(R, 0);
  for (int r = 0; r < R; ++r) {
    gv[r].assign(max_iter + 1, 0.0);
    gv[r][0] = beta[r];
    if (!(beta[r] > 0)) { done[r] = 1; res.rel[r] = 0; }
    H[r].assign(size_t(max_iter + 1) * max_iter, 0.0);
    cs[r].assign(max_iter, 0.0);
    sn[r].assign(max_iter, 0.0);
  }
  std::vector<double2> hh(size_t(max_iter + 1) * R);
  std::vector<double> nr(R);
  int j = 0;
  for (; j < max_iter; ++j) {
    if (std::all_of(done.begin(), done.end(), [](int v) { return v; })) break;
    double2* Vj = d.V_kry + vs * j;
    apply_F(h, Vj, d.t1, R, prec);
    apply_P(h, d.t1, d.w, R, prec);
    int nvec = j + 1;
    HIPCHECK(hipMemsetAsync(d.hsum, 0, size_t(nvec) * R * sizeof(double2), s));
    const double vb = 16.0 * double(vs);
    for (int pass = 0; pass < 2; ++pass) {
      {
        Timed t(h, KF_DOTS, (nvec + 1) * vb, 8.0 * nvec * double(vs));
        launch_dots(d.V_kry, vs, nvec, d.w, n, R, d.part, nblk, s);
        launch_dots_final(d.part, nblk, nvec, R, d.hbuf, d.hsum, s);
      }
      {
        Timed t(h, KF_UPDATE, (nvec + 2) * vb, 8.0 * nvec * double(vs));
        launch_update(d.V_kry, vs, nvec, d.hbuf, d.w, n, R, -1.0, s);
      }
    }
    {
      Timed t(h, KF_NORM_SCALE, 3 * vb, 6.0 * double(vs));
      launch_norm(d.w, n, R, d.npart, nblk, d.nrm, s);
      launch_scale(d.w, d.nrm, d.V_kry + vs * (j + 1), n, R, s);
    }
    HIPCHECK(hipMemcpyAsync(hh.data(), d.hsum, size_t(nvec) * R * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(nr.data(), d.nrm, R * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (int r = 0; r < R; ++r) {
      if (done[r]) continue;
      auto Hc = [&](int i) -> cd& { return H[r][size_t(j) * (max_iter + 1) + i]; };
      for (int i = 0; i < nvec; ++i) Hc(i) = cd(hh[size_t(i) * R + r].x, hh[size_t(i) * R + r].y);
      Hc(j + 1) = nr[r];
      for (int i = 0; i < j; ++i) {
        cd t = cs[r][i] * Hc(i) + sn[r][i] * Hc(i + 1);
        Hc(i + 1) = -std::conj(sn[r][i]) * Hc(i) + cs[r][i] * Hc(i + 1);
        Hc(i) = t;
      }
      cd a = Hc(j), b = Hc(j + 1);
      double den = std::sqrt(std::norm(a) + std::norm(b));
      if (den == 0) { cs[r][j] = 1; sn[r][j] = 0; }
      else if (std::abs(a) == 0) { cs[r][j] = 0; sn[r][j] = std::conj(b) / den; }
      else { cs[r][j] = std::abs(a) / den; sn[r][j] = (a / std::abs(a)) * std::conj(b) / den; }
      Hc(j) = cs[r][j] * a + sn[r][j] * b;
      Hc(j + 1) = 0;
      gv[r][j + 1] = -std::conj(sn[r][j]) * gv[r][j];
      gv[r][j] = cs[r][j] * gv[r][j];
      res.iters[r] = j + 1;
      res.rel[r] = std::abs(gv[r][j + 1]) / beta[r];
      if (res.rel[r] <= tol || nr[r] == 0.0) done[r] = 1;
    }
  }
  // x = sum_i V_i y_i with H y = g (upper triangular, per system)
  std::vector<double2> ycoef(size_t(max_iter + 1) * R, make_double2(0, 0));
  int kmax = 0;
  for (int r = 0; r < R; ++r) {
    int k = res.iters[r];
    kmax = std::max(kmax, k);
    std::vector<cd> y(k);
    for (int i = k - 1; i >= 0; --i) {
      cd sum = gv[r][i];
      for (int jj = i + 1; jj < k; ++jj) sum -= H[r][size_t(jj) * (max_iter + 1) + i] * y[jj];
      y[i] = sum / H[r][size_t(i) * (max_iter + 1) + i];
    }
    for (int i = 0; i < k; ++i) ycoef[size_t(i) * R + r] = make_double2(y[i].real(), y[i].imag());
  }
  if (kmax > 0) {
    HIPCHECK(hipMemcpyAsync(d.ycoef, ycoef.data(), size_t(kmax) * R * sizeof(double2), hipMemcpyHostToDevice, s));
    launch_update(d.V_kry, vs, kmax, d.ycoef, x, n, R, 1.0, s);
  }
  HIPCHECK(hipStreamSynchronize(s));
  return res;
}

}  // namespace hdp

using namespace hdp;

#define API_BEGIN try {
#define API_END                                  \
  }                                              \
  catch (const Error& e) {                       \
    g_err = e.msg;                               \
    return e.status;                             \
  }                                              \
  catch (const std::exception& e) {              \
    g_err = e.what();                            \
    return HDP_E_ARG;                            \
  }

extern "C" {

hdp_status hdp_setup(const hdp_mesh* mesh, const hdp_problem* prob, const hdp_options* opt, hdp_handle** out) {
  API_BEGIN
  if (!out || !opt) fail(HDP_E_ARG, "null output or options");
  *out = nullptr;
  if (opt->max_rhs < 1 || opt->max_rhs > 256) fail(HDP_E_ARG, "max_rhs must lie in 1..256");
  if (opt->max_iter < 1 || opt->max_iter > 2000) fail(HDP_E_ARG, "max_iter must lie in 1..2000");
  if (!(opt->tol > 0) || !(opt->tol < 1)) fail(HDP_E_ARG, "tol must lie in (0,1)");
  if (opt->precision != HDP_FP64 && opt->precision != HDP_MIXED) fail(HDP_E_ARG, "unknown precision");
  auto t0 = std::chrono::steady_clock::now();
  hdp_handle* H = new hdp_handle();
  Handle& h = H->h;
  h.max_rhs = opt->max_rhs;
  h.max_iter = opt->max_iter;
  h.tol = opt->tol;
  h.precision = opt->precision;
  h.stream = static_cast<hipStream_t>(opt->stream);
  try {
    build_host(h, mesh, prob);
    build_device(h);
  } catch (...) {
    for (void* p : h.allocations) (void)hipFree(p);
    delete H;
    throw;
  }
  h.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = H;
  return HDP_OK;
  API_END
}

hdp_status hdp_inspect(const hdp_mesh* mesh, const hdp_problem* prob, hdp_stats* st) {
  API_BEGIN
  if (!st) fail(HDP_E_ARG, "null stats");
  hdp_handle H;
  build_host(H.h, mesh, prob);
  return hdp_get_stats(&H, st);
  API_END
}

hdp_status hdp_get_stats(const hdp_handle* H, hdp_stats* st) {
  API_BEGIN
  if (!H || !st) fail(HDP_E_ARG, "null handle or stats");
  const Handle& h = H->h;
  std::memset(st, 0, sizeof(*st));
  st->dof = h.dof;
  st->n_elements = h.E;
  st->n_lambda = h.nlam;
  st->n_coarse = h.nK;
  st->l = h.l;
  st->n_classes = int(h.classes.size());
  st->min_element_margin = h.min_margin;
  st->setup_ms = h.setup_ms;
  return HDP_OK;
  API_END
}

hdp_status hdp_apply_interface(hdp_handle* H, const hdp_c64* v, hdp_c64* u, int32_t n_rhs, int32_t precision) {
  API_BEGIN
  if (!H || !v || !u) fail(HDP_E_ARG, "null argument");
  Handle& h = H->h;
  if (n_rhs < 1 || n_rhs > pow2ceil(h.max_rhs)) fail(HDP_E_ARG, "n_rhs out of range");
  apply_F(h, reinterpret_cast<const double2*>(v), reinterpret_cast<double2*>(u), n_rhs, precision);
  HIPCHECK(hipStreamSynchronize(h.stream));
  prof_flush(h);
  return HDP_OK;
  API_END
}

hdp_status hdp_apply_precond(hdp_handle* H, const hdp_c64* v, hdp_c64* u, int32_t n_rhs, int32_t precision) {
  API_BEGIN
  if (!H || !v || !u) fail(HDP_E_ARG, "null argument");
  Handle& h = H->h;
  if (n_rhs < 1 || n_rhs > pow2ceil(h.max_rhs)) fail(HDP_E_ARG, "n_rhs out of range");
  apply_P(h, reinterpret_cast<const double2*>(v), reinterpret_cast<double2*>(u), n_rhs, precision);
  HIPCHECK(hipStreamSynchronize(h.stream));
  prof_flush(h);
  return HDP_OK;
  API_END
}

hdp_status hdp_local_solve(hdp_handle* H, const hdp_c64* y, hdp_c64* x, int32_t n_rhs) {
  API_BEGIN
  if (!H || !y || !x) fail(HDP_E_ARG, "null argument");
  Handle& h = H->h;
  if (n_rhs < 1) fail(HDP_E_ARG, "n_rhs out of range");
  launch_fdm(h, reinterpret_cast<const double2*>(y), reinterpret_cast<double2*>(x), n_rhs, h.stream);
  HIPCHECK(hipStreamSynchronize(h.stream));
  return HDP_OK;
  API_END
}

static void check_rhs(const Handle& h, const hdp_rhs* rhs) {
  if (!rhs) fail(HDP_E_ARG, "null rhs");
  if (rhs->n_rhs < 1 || rhs->n_rhs > h.max_rhs) fail(HDP_E_ARG, "n_rhs out of range");
  if (rhs->kind == HDP_RHS_POINT) {
    if (!rhs->points) fail(HDP_E_ARG, "points missing");
    for (int i = 0; i < 2 * rhs->n_rhs; ++i)
      if (!std::isfinite(rhs->points[i])) fail(HDP_E_ARG, "non-finite source point");
  } else if (rhs->kind == HDP_RHS_PLANE_WAVE_TOTAL || rhs->kind == HDP_RHS_PLANE_WAVE_SCATTERED) {
    if (!rhs->angles) fail(HDP_E_ARG, "angles missing");
    for (int i = 0; i < rhs->n_rhs; ++i)
      if (!std::isfinite(rhs->angles[i])) fail(HDP_E_ARG, "non-finite angle");
  } else {
    fail(HDP_E_ARG, "unknown rhs kind");
  }
}

// Loads of all RHS into full0 with stride Rp (zero-padded columns).
static void load_rhs(Handle& h, const hdp_rhs* rhs, int Rp) {
  std::vector<cd> B;
  compute_loads(h, rhs, B);
  int R = rhs->n_rhs;
  std::vector<double2> P(size_t(h.dof) * Rp, make_double2(0, 0));
  for (int64_t i = 0; i < h.dof; ++i)
    for (int r = 0; r < R; ++r) P[size_t(i) * Rp + r] = make_double2(B[size_t(i) * R + r].real(), B[size_t(i) * R + r].imag());
  HIPCHECK(hipMemcpyAsync(h.d.full0, P.data(), P.size() * sizeof(double2), hipMemcpyHostToDevice, h.stream));
  HIPCHECK(hipStreamSynchronize(h.stream));
}

hdp_status hdp_interface_rhs(hdp_handle* H, const hdp_rhs* rhs, hdp_c64* g) {
  API_BEGIN
  if (!H || !g) fail(HDP_E_ARG, "null argument");
  Handle& h = H->h;
  check_rhs(h, rhs);
  int R = rhs->n_rhs;
  load_rhs(h, rhs, R);
  interface_rhs(h, reinterpret_cast<double2*>(g), R);
  HIPCHECK(hipStreamSynchronize(h.stream));
  return HDP_OK;
  API_END
}

hdp_status hdp_solve(hdp_handle* H, const hdp_rhs* rhs, hdp_c64* field, int32_t n_far, const double* far_angles,
                     const uint8_t* far_inside, hdp_c64* far, hdp_stats* stats) {
  API_BEGIN
  if (!H) fail(HDP_E_ARG, "null handle");
  Handle& h = H->h;
  check_rhs(h, rhs);
  if (far && (n_far < 1 || !far_angles || !far_inside)) fail(HDP_E_ARG, "far-field arguments incomplete");
  if (far) fail(HDP_E_UNSUPPORTED, "far field not implemented in this build");
  auto t0 = std::chrono::steady_clock::now();
  auto& d = h.d;
  hipStream_t s = h.stream;
  int R = rhs->n_rhs, Rp = pow2ceil(R);
  int64_t vs = int64_t(h.nlam) * Rp;
  load_rhs(h, rhs, Rp);
  interface_rhs(h, d.t0, Rp);                       // g
  int iters = 0, refinements = 0;
  double rel = 0;
  bool conv = true;
  if (h.precision == HDP_FP64) {
    GmresResult gr = gmres(h, d.t0, d.t2, Rp, HDP_FP64, h.tol, h.max_iter);
    for (int r = 0; r < R; ++r) {
      iters = std::max(iters, gr.iters[r]);
      rel = std::max(rel, gr.rel[r]);
      if (gr.rel[r] > h.tol) conv = false;
    }
  } else {
    // GMRES-IR: inner GMRES on FP32 local operators, FP64 residual and update
    int nblk = dots_blocks(h.nlam, Rp);
    HIPCHECK(hipMemsetAsync(d.t2, 0, size_t(vs) * sizeof(double2), s));
    apply_P(h, d.t0, d.w, Rp, HDP_FP64);
    launch_norm(d.w, h.nlam, Rp, d.npart, nblk, d.nrm, s);
    std::vector<double> s0(Rp), sk(Rp);
    HIPCHECK(hipMemcpyAsync(s0.data(), d.nrm, Rp * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    HIPCHECK(hipMemcpyAsync(d.t1, d.t0, size_t(vs) * sizeof(double2), hipMemcpyDeviceToDevice, s));  // r = g
    double2* delta = nullptr;
    delta = d.full1;   // scratch of at least nlam * Rp (dof >= nlam)
    int budget = h.max_iter;
    conv = false;
    for (int outer = 0; outer < 30 && budget > 0; ++outer) {
      GmresResult gr = gmres(h, d.t1, delta, Rp, HDP_MIXED, 1e-5, budget);
      int used = 0;
      for (int r = 0; r < R; ++r) used = std::max(used, gr.iters[r]);
      iters += used;
      budget -= std::max(used, 1);
      ++refinements;
      launch_axpby(d.t2, delta, d.t2, vs, 1.0, 1.0, s);   // nu += delta
      apply_F(h, d.t2, d.t1, Rp, HDP_FP64);                // F nu
      launch_axpby(d.t0, d.t1, d.t1, vs, 1.0, -1.0, s);   // r = g - F nu
      apply_P(h, d.t1, d.w, Rp, HDP_FP64);
      launch_norm(d.w, h.nlam, Rp, d.npart, nblk, d.nrm, s);
      HIPCHECK(hipMemcpyAsync(sk.data(), d.nrm, Rp * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      rel = 0;
      for (int r = 0; r < R; ++r) rel = std::max(rel, s0[r] > 0 ? sk[r] / s0[r] : 0.0);
      if (rel <= h.tol) { conv = true; break; }
    }
  }
  // recovery phi = A^-1 (b^ - C^T nu) (Sec. 2.3.1) and the field at GLL nodes
  HIPCHECK(hipMemcpyAsync(d.full1, d.full0, size_t(h.dof) * Rp * sizeof(double2), hipMemcpyDeviceToDevice, s));
  launch_sub_dual(h, d.full1, d.t2, Rp, s);
  element_solve(h, d.full1, d.full0, Rp);
  if (field) {
    Timed t(h, KF_GLL, 2.0 * h.dof * 16.0 * R, h.flops_gll * R);
    launch_gll(h, d.full1, reinterpret_cast<double2*>(field), Rp, h.dof, R, s);
  }
  HIPCHECK(hipStreamSynchronize(s));
  prof_flush(h);
  double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) {
    hdp_get_stats(H, stats);
    stats->iterations = iters;
    stats->refinements = refinements;
    stats->rel_residual = rel;
    stats->solve_ms = ms;
  }
  return conv ? HDP_OK : HDP_W_NOT_CONVERGED;
  API_END
}

hdp_status hdp_profile(hdp_handle* H, int32_t enable) {
  API_BEGIN
  if (!H) fail(HDP_E_ARG, "null handle");
  Handle& h = H->h;
  HIPCHECK(hipStreamSynchronize(h.stream));
  prof_flush(h);
  if (enable) {
    for (int f = 0; f < KF_COUNT; ++f) h.prof.ms[f] = h.prof.bytes[f] = h.prof.flops[f] = 0, h.prof.n[f] = 0;
  }
  h.prof.on = enable != 0;
  return HDP_OK;
  API_END
}

hdp_status hdp_profile_read(const hdp_handle* H, hdp_kernel_time* out, int32_t max, int32_t* count) {
  API_BEGIN
  if (!H || !count) fail(HDP_E_ARG, "null argument");
  const Handle& h = H->h;
  *count = KF_COUNT;
  for (int f = 0; f < KF_COUNT && f < max && out; ++f) {
    std::memset(&out[f], 0, sizeof(out[f]));
    std::strncpy(out[f].name, KF_NAMES[f], sizeof(out[f].name) - 1);
    out[f].launches = h.prof.n[f];
    out[f].total_ms = h.prof.ms[f];
    out[f].bytes = h.prof.bytes[f];
    out[f].flops = h.prof.flops[f];
  }
  return HDP_OK;
  API_END
}

void hdp_destroy(hdp_handle* H) {
  if (!H) return;
  if (H->h.stream) (void)hipStreamSynchronize(H->h.stream);
  else (void)hipDeviceSynchronize();
  for (auto& p : H->h.prof.pend) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : H->h.prof.pool) (void)hipEventDestroy(e);
  for (void* p : H->h.allocations) (void)hipFree(p);
  delete H;
}

const char* hdp_status_string(hdp_status s) {
  switch (s) {
    case HDP_OK: return "ok";
    case HDP_W_NOT_CONVERGED: return "not converged";
    case HDP_E_ARG: return "invalid argument";
    case HDP_E_MESH: return "invalid mesh";
    case HDP_E_RESONANCE: return "element resonance";
    case HDP_E_COARSE: return "singular coarse matrix";
    case HDP_E_DEVICE: return "device error";
    case HDP_E_NOMEM: return "out of device memory";
    case HDP_E_UNSUPPORTED: return "unsupported input";
  }
  return "unknown status";
}

const char* hdp_last_error_detail(void) { return g_err.c_str(); }

}  // extern "C"
