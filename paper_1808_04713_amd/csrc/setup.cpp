// Host-side setup: mesh analysis, element classes, separable eigenbases,
// per-class boundary operators, dual-row and coarse numbering, loads.
// Paper Sec. 2.2.1 (element matrices), Sec. 2.2.4 (edge constraints),
// Sec. 2.3.2 (Algorithm 1), Sec. 2.3.3 (block structure and preconditioner).
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

#include "basis.hpp"
#include "internal.hpp"

namespace hdp {

namespace {

const double SQ2 = std::sqrt(2.0);

// Local flat mode index of bubble k on a side (vertex basis: along x, index 0
// is the vertex function at x=+1 and index 1 the one at x=-1).
inline int side_mode(int n, int side, int k) {
  switch (side) {
    case 1: return 1 + n * k;   // left  (x = -1)
    case 2: return 0 + n * k;   // right (x = +1)
    case 3: return k + n * 1;   // bottom (y = -1)
    default: return k + n * 0;  // top (y = +1)
  }
}

struct SideKey {
  int kind;          // 0 vertical line, 1 horizontal line
  int64_t c, lo, hi;
  bool operator<(const SideKey& o) const {
    return std::tie(kind, c, lo, hi) < std::tie(o.kind, o.c, o.lo, o.hi);
  }
};

// Separable fast solver on the host: X = Ex [(Ex^T Y Ey) ./ Dg] Ey^T.
MatC fdm_host(const ElemClass& C, const MatC& Y) {
  MatC T = matmul(transpose(C.Ex), Y);
  T = matmul(T, C.Ey);
  for (int j = 0; j < C.n; ++j)
    for (int i = 0; i < C.n; ++i) T(i, j) /= C.Dg[i + C.n * j];
  T = matmul(C.Ex, T);
  return matmul(T, transpose(C.Ey));
}

// Generalised eigenpairs A E = M E Lambda with E^T M E = I (transpose, not
// conjugate: the pencil is complex symmetric), M real SPD.
void gen_eig(const MatC& A, const MatD& M, MatC& E, std::vector<cd>& lam) {
  int n = A.r;
  MatD L = cholesky(M);
  MatD Li = inverse(L);
  MatC Lic = to_complex(Li);
  MatC Cm = matmul(matmul(Lic, A), transpose(Lic));
  bool real = true;
  for (auto& v : Cm.a) if (v.imag() != 0.0) { real = false; break; }
  MatC Q(n, n);
  lam.assign(n, 0);
  if (real) {
    MatD Cr(n, n);
    for (size_t i = 0; i < Cm.a.size(); ++i) Cr.a[i] = Cm.a[i].real();
    std::vector<double> w;
    MatD V;
    jacobi_eig(Cr, w, V);
    for (int j = 0; j < n; ++j) {
      lam[j] = w[j];
      for (int i = 0; i < n; ++i) Q(i, j) = V(i, j);
    }
  } else {
    // symmetrise exactly before the general solver
    for (int j = 0; j < n; ++j)
      for (int i = j + 1; i < n; ++i) {
        cd s = 0.5 * (Cm(i, j) + Cm(j, i));
        Cm(i, j) = Cm(j, i) = s;
      }
    MatC X;
    complex_eig(Cm, lam, X);
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int i = 0; i < n; ++i) s += X(i, j) * X(i, j);
      cd r = std::sqrt(s);
      if (std::abs(r) < 1e-300) fail(HDP_E_RESONANCE, "eigenvector with zero bilinear norm");
      for (int i = 0; i < n; ++i) Q(i, j) = X(i, j) / r;
    }
  }
  E = matmul(transpose(Lic), Q);
  // verify E^T M E = I and E^T A E = diag(lam)
  MatC EtME = matmul(matmul(transpose(E), to_complex(M)), E);
  MatC EtAE = matmul(matmul(transpose(E), A), E);
  double scale = 0;
  for (auto& v : lam) scale = std::max(scale, std::abs(v));
  double err1 = 0, err2 = 0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      err1 = std::max(err1, std::abs(EtME(i, j) - (i == j ? 1.0 : 0.0)));
      err2 = std::max(err2, std::abs(EtAE(i, j) - (i == j ? lam[i] : cd(0))));
    }
  if (err1 > 1e-8 || err2 > 1e-8 * std::max(scale, 1.0))
    fail(HDP_E_RESONANCE, "separable eigenbasis is ill-conditioned (defective 1-D pencil)");
}

void build_class(ElemClass& C, double k, int l) {
  int n = C.n, p = C.p;
  C.nr = 4 * l;
  MatD Mt = mass_vertex(n), Kt = stiffness_vertex(n);
  cd gamma(0.0, -k);
  double beta = -k * k * C.eps;
  MatC Ax(n, n), Ay(n, n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      Ax(i, j) = (2.0 / C.hx) * Kt(i, j) + beta * (C.hx / 2.0) * Mt(i, j);
      Ay(i, j) = (2.0 / C.hy) * Kt(i, j);
    }
  // Robin terms gamma * |J_edge| * (trace mode)(trace mode)^T on boundary sides
  if (C.bmask & 1) Ax(1, 1) += gamma;   // left: vertex mode at x=-1
  if (C.bmask & 2) Ax(0, 0) += gamma;   // right
  if (C.bmask & 4) Ay(1, 1) += gamma;   // bottom
  if (C.bmask & 8) Ay(0, 0) += gamma;   // top
  std::vector<cd> lx, ly;
  gen_eig(Ax, Mt, C.Ex, lx);
  gen_eig(Ay, Mt, C.Ey, ly);
  C.Dg.assign(n * n, 0);
  double mn = 1e300, mx = 0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      cd d = (C.hy / 2.0) * lx[i] + (C.hx / 2.0) * ly[j];
      C.Dg[i + n * j] = d;
      mn = std::min(mn, std::abs(d));
      mx = std::max(mx, std::abs(d));
    }
  C.margin = mn / mx;
  if (!(C.margin > 1e-13)) fail(HDP_E_RESONANCE, "element matrix singular at this wavenumber");
  // coarse modes: vertices, then bubbles 2..l on sides left, right, bottom, top
  C.R = {1 + n, 0 + n, 1, 0};
  for (int s = 1; s <= 4; ++s)
    for (int kk = 2; kk <= l; ++kk) C.R.push_back(side_mode(n, s, kk));
  C.Gam.clear();
  for (int s = 1; s <= 4; ++s) {
    if (C.bmask & (1 << (s - 1))) continue;
    for (int kk = l + 1; kk <= p; ++kk) C.Gam.push_back(side_mode(n, s, kk));
  }
  C.m = int(C.Gam.size());
  int nr = C.nr, m = C.m, n2 = n * n;
  auto unit_solve = [&](int mode) {
    MatC Y(n, n);
    Y.a[mode] = 1.0;
    return fdm_host(C, Y);
  };
  C.G = MatC(n2, nr);
  for (int r = 0; r < nr; ++r) {
    MatC X = unit_solve(C.R[r]);
    for (int i = 0; i < n2; ++i) C.G(i, r) = X.a[i];
  }
  MatC Ccap(nr, nr);
  for (int b = 0; b < nr; ++b)
    for (int a = 0; a < nr; ++a) Ccap(a, b) = C.G(C.R[a], b);
  // C_cap is the coarse block of A~^-1; its inverse is the element coarse matrix
  try {
    C.Kc = inverse(Ccap);
  } catch (...) {
    fail(HDP_E_RESONANCE, "element coarse block singular");
  }
  MatC H(m, m), GG(m, nr);
  for (int g = 0; g < m; ++g) {
    MatC X = unit_solve(C.Gam[g]);
    for (int a = 0; a < m; ++a) H(a, g) = X.a[C.Gam[a]];
    for (int r = 0; r < nr; ++r) GG(g, r) = C.G(C.Gam[g], r);
  }
  MatC GK = matmul(GG, C.Kc);          // G_Gam Kc
  C.Phi = MatC(m, nr);
  for (int r = 0; r < nr; ++r)
    for (int a = 0; a < m; ++a) C.Phi(a, r) = -GK(a, r);
  MatC Dc = matmul(GK, transpose(GG));
  for (size_t i = 0; i < Dc.a.size(); ++i) Dc.a[i] = H.a[i] - Dc.a[i];
  C.Op1 = MatC(m + nr, m);
  for (int b = 0; b < m; ++b) {
    for (int a = 0; a < m; ++a) C.Op1(a, b) = Dc(a, b);
    for (int r = 0; r < nr; ++r) C.Op1(m + r, b) = C.Phi(b, r);
  }
  // Laplace-only Dirichlet preconditioner block: Schur complement of A~_L
  // restricted to the type-1 set onto its edge modes (interior eliminated).
  std::vector<int> inR(n2, 0);
  for (int r : C.R) inR[r] = 1;
  std::vector<int> emodes, imodes;
  for (int md = 0; md < n2; ++md) {
    if (inR[md]) continue;
    int ix = md % n, iy = md / n;
    if (ix >= 2 && iy >= 2) imodes.push_back(md);
    else emodes.push_back(md);
  }
  auto AL = [&](int a, int b) {
    int i1 = a % n, i2 = a / n, j1 = b % n, j2 = b / n;
    return (C.hy / C.hx) * Mt(i2, j2) * Kt(i1, j1) + (C.hx / C.hy) * Kt(i2, j2) * Mt(i1, j1);
  };
  int ne = int(emodes.size()), ni = int(imodes.size());
  MatD Aee(ne, ne), Aei(ne, ni), Aii(ni, ni);
  for (int b = 0; b < ne; ++b)
    for (int a = 0; a < ne; ++a) Aee(a, b) = AL(emodes[a], emodes[b]);
  for (int b = 0; b < ni; ++b)
    for (int a = 0; a < ne; ++a) Aei(a, b) = AL(emodes[a], imodes[b]);
  for (int b = 0; b < ni; ++b)
    for (int a = 0; a < ni; ++a) Aii(a, b) = AL(imodes[a], imodes[b]);
  MatD S = Aee;
  if (ni > 0) {
    MatD X = solve(Aii, transpose(Aei));
    MatD AX = matmul(Aei, X);
    for (size_t i = 0; i < S.a.size(); ++i) S.a[i] -= AX.a[i];
  }
  std::vector<int> epos(n2, -1);
  for (int a = 0; a < ne; ++a) epos[emodes[a]] = a;
  C.Se = MatD(m, m);
  for (int b = 0; b < m; ++b)
    for (int a = 0; a < m; ++a) C.Se(a, b) = S(epos[C.Gam[a]], epos[C.Gam[b]]);
}

}  // namespace

void build_host(Handle& h, const hdp_mesh* mesh, const hdp_problem* prob) {
  if (!mesh || !prob || !mesh->leaf || !mesh->degree) fail(HDP_E_ARG, "null mesh or problem");
  int E = mesh->n_leaves;
  if (E <= 0 || mesh->base_nx <= 0 || mesh->base_ny <= 0) fail(HDP_E_ARG, "empty mesh");
  if (!(mesh->x1 > mesh->x0) || !(mesh->y1 > mesh->y0)) fail(HDP_E_ARG, "bad domain");
  if (!(prob->k > 0) || !std::isfinite(prob->k)) fail(HDP_E_ARG, "k must be positive and finite");
  h.E = E;
  h.k = prob->k;
  int Lmax = 0;
  for (int e = 0; e < E; ++e) {
    int lev = mesh->leaf[3 * e];
    if (lev < 0 || lev > 20) fail(HDP_E_MESH, "leaf level out of range");
    Lmax = std::max(Lmax, lev);
  }
  int64_t NX = int64_t(mesh->base_nx) << Lmax, NY = int64_t(mesh->base_ny) << Lmax;
  double fhx = (mesh->x1 - mesh->x0) / double(NX), fhy = (mesh->y1 - mesh->y0) / double(NY);
  std::vector<int64_t> X0(E), X1(E), Y0(E), Y1(E);
  std::vector<int> level(E);
  h.deg.resize(E);
  h.eps.assign(E, 1.0);
  h.ox.resize(E); h.oy.resize(E); h.hx.resize(E); h.hy.resize(E);
  int64_t area = 0;
  for (int e = 0; e < E; ++e) {
    int lev = mesh->leaf[3 * e], ix = mesh->leaf[3 * e + 1], iy = mesh->leaf[3 * e + 2];
    if (ix < 0 || iy < 0 || ix >= (mesh->base_nx << lev) || iy >= (mesh->base_ny << lev))
      fail(HDP_E_MESH, "leaf index outside the base grid");
    int64_t s = int64_t(1) << (Lmax - lev);
    X0[e] = ix * s; X1[e] = (ix + 1) * s; Y0[e] = iy * s; Y1[e] = (iy + 1) * s;
    area += s * s;
    level[e] = lev;
    int p = mesh->degree[e];
    if (p < 1 || p > 40) fail(HDP_E_ARG, "degree must lie in 1..40");
    h.deg[e] = p;
    if (prob->eps_r) {
      h.eps[e] = prob->eps_r[e];
      if (!std::isfinite(h.eps[e])) fail(HDP_E_ARG, "eps_r not finite");
    }
    h.ox[e] = mesh->x0 + X0[e] * fhx;
    h.oy[e] = mesh->y0 + Y0[e] * fhy;
    h.hx[e] = s * fhx;
    h.hy[e] = s * fhy;
  }
  if (area != NX * NY) fail(HDP_E_MESH, "leaves do not tile the domain");
  // sides: match interior sides pairwise (conforming meshes only)
  std::map<SideKey, std::vector<std::pair<int, int>>> sides;
  auto key_of = [&](int e, int s) {
    switch (s) {
      case 1: return SideKey{0, X0[e], Y0[e], Y1[e]};
      case 2: return SideKey{0, X1[e], Y0[e], Y1[e]};
      case 3: return SideKey{1, Y0[e], X0[e], X1[e]};
      default: return SideKey{1, Y1[e], X0[e], X1[e]};
    }
  };
  for (int e = 0; e < E; ++e)
    for (int s = 1; s <= 4; ++s) sides[key_of(e, s)].push_back({e, s});
  std::vector<int> nb_e(4 * E, -1), nb_s(4 * E, 0);
  h.bmask.assign(E, 0);
  for (int e = 0; e < E; ++e)
    for (int s = 1; s <= 4; ++s) {
      SideKey key = key_of(e, s);
      bool bnd = (key.kind == 0 && (key.c == 0 || key.c == NX)) ||
                 (key.kind == 1 && (key.c == 0 || key.c == NY));
      if (bnd) { h.bmask[e] |= 1 << (s - 1); continue; }
      auto& v = sides[key];
      if (v.size() != 2)
        fail(HDP_E_UNSUPPORTED, "non-conforming (hanging) edges are not supported by this build");
      auto o = v[0].first == e ? v[1] : v[0];
      if (o.first == e) fail(HDP_E_MESH, "duplicate leaf");
      nb_e[4 * e + s - 1] = o.first;
      nb_s[4 * e + s - 1] = o.second;
    }
  h.nb_e = nb_e;
  // coarse order l (Sec. 2.3.4): the criterion is evaluated for every element with
  // its longest edge and its local wavenumber k sqrt(eps_r), and the largest value
  // is used (with eps_r = 1 this is the free-space k and the longest edge)
  double khmax = 0;
  for (int e = 0; e < E; ++e)
    khmax = std::max(khmax, prob->k * std::sqrt(std::max(h.eps[e], 0.0)) * std::max(h.hx[e], h.hy[e]));
  h.l = prob->l > 0 ? prob->l : dispersion_l(khmax, 1.0) + std::max(0, prob->l_safety);
  for (int e = 0; e < E; ++e)
    if (h.l >= h.deg[e])
      fail(HDP_E_UNSUPPORTED, "coarse order l must be below every element degree in this build");
  int l = h.l;
  // classes
  std::map<std::tuple<int, double, double, double, int>, int> cmap;
  h.cls.resize(E);
  for (int e = 0; e < E; ++e) {
    auto key = std::make_tuple(h.deg[e], h.hx[e], h.hy[e], h.eps[e], h.bmask[e]);
    auto it = cmap.find(key);
    if (it == cmap.end()) {
      ElemClass C;
      C.p = h.deg[e]; C.n = C.p + 1; C.hx = h.hx[e]; C.hy = h.hy[e];
      C.eps = h.eps[e]; C.bmask = h.bmask[e];
      it = cmap.emplace(key, int(h.classes.size())).first;
      h.classes.push_back(C);
    }
    h.cls[e] = it->second;
    h.classes[it->second].elems.push_back(e);
  }
  h.min_margin = 1;
  for (auto& C : h.classes) {
    build_class(C, h.k, l);
    h.min_margin = std::min(h.min_margin, C.margin);
  }
  // offsets
  h.dof_off.assign(E + 1, 0);
  h.slot_off.assign(E + 1, 0);
  h.cm_off.assign(E + 1, 0);
  for (int e = 0; e < E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    h.dof_off[e + 1] = h.dof_off[e] + int64_t(C.n) * C.n;
    h.slot_off[e + 1] = h.slot_off[e] + C.m;
    h.cm_off[e + 1] = h.cm_off[e] + C.nr;
  }
  h.dof = h.dof_off[E];
  h.nslots = h.slot_off[E];
  h.ncm = h.cm_off[E];
  // slot lookup: (element, side, k) -> global slot
  auto slot_of = [&](int e, int s, int kk) {
    const ElemClass& C = h.classes[h.cls[e]];
    int pos = 0;
    for (int t = 1; t < s; ++t)
      if (!(C.bmask & (1 << (t - 1)))) pos += C.p - l;
    return h.slot_off[e] + pos + (kk - l - 1);
  };
  // dual rows in Algorithm 1 visiting order
  std::vector<int> vorder(E);
  for (int e = 0; e < E; ++e) vorder[e] = e;
  std::stable_sort(vorder.begin(), vorder.end(), [&](int a, int b) { return level[a] > level[b]; });
  std::vector<char> visited(4 * E, 0);
  h.row_slot.clear(); h.row_coef.clear();
  h.slot_row.assign(h.nslots, -1);
  h.slot_coef.assign(h.nslots, 0.0);
  h.slot_mode.assign(h.nslots, 0);
  for (int e : vorder)
    for (int s = 1; s <= 4; ++s) {
      if (h.bmask[e] & (1 << (s - 1))) continue;
      if (visited[4 * e + s - 1]) continue;
      int c = nb_e[4 * e + s - 1], sc = nb_s[4 * e + s - 1];
      visited[4 * e + s - 1] = visited[4 * c + sc - 1] = 1;
      int L = std::max(h.deg[e], h.deg[c]);
      for (int kk = l + 1; kk <= L; ++kk) {
        int row = int(h.row_coef.size() / 2);
        int a = kk <= h.deg[c] ? slot_of(c, sc, kk) : -1;
        int b = kk <= h.deg[e] ? slot_of(e, s, kk) : -1;
        h.row_slot.push_back(a);
        h.row_coef.push_back(a >= 0 ? SQ2 : 0.0);
        h.row_slot.push_back(b);
        h.row_coef.push_back(b >= 0 ? -SQ2 : 0.0);
        if (a >= 0) { h.slot_row[a] = row; h.slot_coef[a] = SQ2; }
        if (b >= 0) { h.slot_row[b] = row; h.slot_coef[b] = -SQ2; }
      }
    }
  h.nlam = int(h.row_coef.size() / 2);
  h.row_xinv.resize(h.nlam);
  for (int r = 0; r < h.nlam; ++r) {
    double x = h.row_coef[2 * r] * h.row_coef[2 * r] + h.row_coef[2 * r + 1] * h.row_coef[2 * r + 1];
    h.row_xinv[r] = 1.0 / x;
  }
  for (int e = 0; e < E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    for (int g = 0; g < C.m; ++g) {
      h.slot_mode[h.slot_off[e] + g] = C.Gam[g];
      if (h.slot_row[h.slot_off[e] + g] < 0) fail(HDP_E_MESH, "dual slot without a row");
    }
  }
  // coarse unknowns: one per mesh vertex and per low-order bubble of every edge
  std::map<std::tuple<int, int64_t, int64_t, int64_t, int>, int> cids;
  h.cm_dof.assign(h.ncm, -1);
  h.cm_mode.assign(h.ncm, 0);
  for (int e = 0; e < E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    int64_t vx[2] = {X1[e], X0[e]}, vy[2] = {Y1[e], Y0[e]};
    for (int r = 0; r < C.nr; ++r) {
      int md = C.R[r], n = C.n, ix = md % n, iy = md / n;
      std::tuple<int, int64_t, int64_t, int64_t, int> key;
      if (ix < 2 && iy < 2) {
        key = std::make_tuple(-1, vx[ix], vy[iy], int64_t(0), 0);
      } else {
        int s, kk;
        if (ix == 0) { s = 2; kk = iy; }
        else if (ix == 1) { s = 1; kk = iy; }
        else if (iy == 0) { s = 4; kk = ix; }
        else { s = 3; kk = ix; }
        SideKey sk = key_of(e, s);
        key = std::make_tuple(sk.kind, sk.c, sk.lo, sk.hi, kk);
      }
      auto it = cids.find(key);
      if (it == cids.end()) it = cids.emplace(key, int(cids.size())).first;
      h.cm_dof[h.cm_off[e] + r] = it->second;
      h.cm_mode[h.cm_off[e] + r] = md;
    }
  }
  h.nK = int(cids.size());
  h.cdof_ptr.assign(h.nK + 1, 0);
  for (int i = 0; i < h.ncm; ++i) h.cdof_ptr[h.cm_dof[i] + 1]++;
  for (int i = 0; i < h.nK; ++i) h.cdof_ptr[i + 1] += h.cdof_ptr[i];
  h.cdof_list.assign(h.ncm, 0);
  std::vector<int> fill(h.cdof_ptr.begin(), h.cdof_ptr.end() - 1);
  for (int i = 0; i < h.ncm; ++i) h.cdof_list[fill[h.cm_dof[i]]++] = i;
  // algorithmic work counts
  for (auto& C : h.classes) {
    h.op1_bytes += 16.0 * (C.m + C.nr) * C.m;
    h.se_bytes += 8.0 * C.m * C.m;
    h.phi_bytes += 16.0 * C.m * C.nr;
  }
  for (int e = 0; e < E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    h.flops_F += 8.0 * (C.m + C.nr) * C.m;
    h.flops_P += 4.0 * C.m * C.m;
    h.flops_coarse += 8.0 * C.m * C.nr;
    h.flops_fdm += 4.0 * 8.0 * double(C.n) * C.n * C.n;
    h.flops_gll += 2.0 * 4.0 * double(C.n) * C.n * C.n;
  }
  // quadrature tables for the loads, one per degree present
  for (auto& C : h.classes) {
    if (h.quad_x.count(C.n)) continue;
    std::vector<double> xq, wq;
    gauss_legendre(C.n + 40, xq, wq);
    std::vector<double> Nq(xq.size() * C.n);
    for (size_t t = 0; t < xq.size(); ++t) vertex_basis(C.n, xq[t], &Nq[t * C.n]);
    h.quad_x[C.n] = xq;
    h.quad_w[C.n] = wq;
    h.quad_N[C.n] = Nq;
  }
  // class-grouped element order
  h.order.clear();
  for (auto& C : h.classes)
    for (int e : C.elems) h.order.push_back(e);
}

// Element loads b~_e in the vertex basis (Sec. 2.2.1: f~ and r_i), only for
// elements whose load is non-zero.
void compute_loads(const Handle& h, const hdp_rhs* rhs, int R, std::vector<int>& elems, std::vector<cd>& vals) {
  elems.clear();
  vals.clear();
  const int nr = rhs->n_rhs;
  double k = h.k;
  cd I(0, 1);
  // owners of each point source (equal split among the elements whose closure holds it)
  std::vector<std::vector<int>> owners(nr);
  if (rhs->kind == HDP_RHS_POINT) {
    for (int r = 0; r < nr; ++r) {
      double px = rhs->points[2 * r], py = rhs->points[2 * r + 1];
      double tol = 1e-12 * std::max(1.0, std::max(std::abs(px), std::abs(py)));
      for (int f = 0; f < h.E; ++f)
        if (px >= h.ox[f] - tol && px <= h.ox[f] + h.hx[f] + tol && py >= h.oy[f] - tol &&
            py <= h.oy[f] + h.hy[f] + tol)
          owners[r].push_back(f);
    }
  }
  std::vector<char> touched(h.E, 0);
  if (rhs->kind == HDP_RHS_POINT) {
    for (auto& o : owners)
      for (int f : o) touched[f] = 1;
  } else if (rhs->kind == HDP_RHS_PLANE_WAVE_TOTAL) {
    for (int e = 0; e < h.E; ++e) touched[e] = h.bmask[e] != 0;
  } else if (rhs->kind == HDP_RHS_PLANE_WAVE_SCATTERED) {
    for (int e = 0; e < h.E; ++e) touched[e] = h.eps[e] != 1.0;
  } else {
    fail(HDP_E_ARG, "unknown right-hand-side kind");
  }
  for (int e = 0; e < h.E; ++e) {
    if (!touched[e]) continue;
    int n = h.deg[e] + 1;
    const std::vector<double>& xq = h.quad_x.at(n);
    const std::vector<double>& wq = h.quad_w.at(n);
    const std::vector<double>& Nq = h.quad_N.at(n);
    int q = int(xq.size());
    double hx = h.hx[e], hy = h.hy[e], ox = h.ox[e], oy = h.oy[e];
    size_t base = vals.size();
    elems.push_back(e);
    vals.resize(base + size_t(n) * n * R, 0.0);
    auto at = [&](int ix, int iy, int r) -> cd& { return vals[base + (ix + size_t(n) * iy) * R + r]; };
    for (int r = 0; r < nr; ++r) {
      if (rhs->kind == HDP_RHS_PLANE_WAVE_TOTAL) {
        double th = rhs->angles[r], dx = std::cos(th), dy = std::sin(th);
        for (int s = 1; s <= 4; ++s) {
          if (!(h.bmask[e] & (1 << (s - 1)))) continue;
          double nx = s == 1 ? -1 : s == 2 ? 1 : 0, ny = s == 3 ? -1 : s == 4 ? 1 : 0;
          double hl = s <= 2 ? hy : hx;
          std::vector<cd> v(n, 0.0);
          for (int t = 0; t < q; ++t) {
            double x, y;
            if (s <= 2) { x = s == 1 ? ox : ox + hx; y = oy + (xq[t] + 1) * hy / 2; }
            else { y = s == 3 ? oy : oy + hy; x = ox + (xq[t] + 1) * hx / 2; }
            cd g = I * k * (dx * nx + dy * ny - 1.0) * std::exp(I * k * (dx * x + dy * y));
            for (int mm = 0; mm < n; ++mm) v[mm] += wq[t] * (hl / 2) * g * Nq[size_t(t) * n + mm];
          }
          for (int mm = 0; mm < n; ++mm) {
            if (s == 1) at(1, mm, r) += v[mm];
            else if (s == 2) at(0, mm, r) += v[mm];
            else if (s == 3) at(mm, 1, r) += v[mm];
            else at(mm, 0, r) += v[mm];
          }
        }
      } else if (rhs->kind == HDP_RHS_PLANE_WAVE_SCATTERED) {
        double th = rhs->angles[r], dx = std::cos(th), dy = std::sin(th);
        std::vector<cd> a(n, 0.0), b(n, 0.0);
        for (int t = 0; t < q; ++t) {
          double x = ox + (xq[t] + 1) * hx / 2, y = oy + (xq[t] + 1) * hy / 2;
          cd ex = std::exp(I * k * dx * x), ey = std::exp(I * k * dy * y);
          for (int mm = 0; mm < n; ++mm) {
            a[mm] += wq[t] * ex * Nq[size_t(t) * n + mm];
            b[mm] += wq[t] * ey * Nq[size_t(t) * n + mm];
          }
        }
        double f0 = k * k * (h.eps[e] - 1.0) * (hx / 2) * (hy / 2);
        for (int iy = 0; iy < n; ++iy)
          for (int ix = 0; ix < n; ++ix) at(ix, iy, r) += f0 * a[ix] * b[iy];
      } else {
        const auto& o = owners[r];
        if (std::find(o.begin(), o.end(), e) == o.end()) continue;
        double px = rhs->points[2 * r], py = rhs->points[2 * r + 1];
        double u = std::clamp(2 * (px - ox) / hx - 1, -1.0, 1.0);
        double v = std::clamp(2 * (py - oy) / hy - 1, -1.0, 1.0);
        std::vector<double> Nu(n), Nv(n);
        vertex_basis(n, u, Nu.data());
        vertex_basis(n, v, Nv.data());
        for (int iy = 0; iy < n; ++iy)
          for (int ix = 0; ix < n; ++ix) at(ix, iy, r) += Nu[ix] * Nv[iy] / double(o.size());
      }
    }
  }
}

}  // namespace hdp
