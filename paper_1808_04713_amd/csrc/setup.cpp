// Host-side setup: mesh analysis, element classes, separable eigenbases,
// per-class boundary operators, dual-row and coarse numbering, loads.
// Paper Sec. 2.2.1 (element matrices), Sec. 2.2.4 (edge constraints),
// Sec. 2.3.2 (Algorithm 1), Sec. 2.3.3 (block structure and preconditioner).
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <exception>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <thread>
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

void build_class(ElemClass& C, double k) {
  int n = C.n, p = C.p;
  MatD Mt = mass_vertex(n), Kt = stiffness_vertex(n);
  cd gamma(0.0, -k);
  // layers (Sec. 3.3): s = 1 + i sigma / k per axis, alpha = diag(s_y/s_x, s_x/s_y),
  // beta = -k^2 eps s_x s_y (all 1 and real outside the layers)
  const cd sx(1.0, C.sigx / k), sy(1.0, C.sigy / k);
  const cd axx = sy / sx, ayy = sx / sy;
  const cd beta = -k * k * C.eps * sx * sy;
  MatC Ax(n, n), Ay(n, n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      Ax(i, j) = axx * (2.0 / C.hx) * Kt(i, j) + beta * (C.hx / 2.0) * Mt(i, j);
      Ay(i, j) = ayy * (2.0 / C.hy) * Kt(i, j);
    }
  // Robin terms gamma * |J_edge| * (trace mode)(trace mode)^T: gamma = -ik on the
  // impedance boundary, +-ik on Robin-modified interior sides (Sec. 2.3.4)
  auto side_gamma = [&](int s) -> cd {
    if (C.bmask & (1 << (s - 1))) return gamma;
    const int code = (C.rmask >> (2 * (s - 1))) & 3;
    return code == 1 ? cd(0.0, -k) : code == 2 ? cd(0.0, k) : cd(0.0, 0.0);
  };
  Ax(1, 1) += side_gamma(1);   // left: vertex mode at x=-1
  Ax(0, 0) += side_gamma(2);   // right
  Ay(1, 1) += side_gamma(3);   // bottom
  Ay(0, 0) += side_gamma(4);   // top
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
  // coarse modes: vertices, then on sides left, right, bottom, top the bubbles
  // 2..top (top: the side's primal count, or p on the coarse side of a hanging edge)
  C.R = {1 + n, 0 + n, 1, 0};
  for (int s = 1; s <= 4; ++s)
    for (int kk = 2; kk <= C.top[s - 1]; ++kk) C.R.push_back(side_mode(n, s, kk));
  C.nr = int(C.R.size());
  // dual slots: the bubbles top+1..gtop of every side (none on the outer boundary;
  // above gtop only where decayed hanging-edge constraints were dropped)
  C.Gam.clear();
  for (int s = 1; s <= 4; ++s)
    for (int kk = C.top[s - 1] + 1; kk <= C.gtop[s - 1]; ++kk) C.Gam.push_back(side_mode(n, s, kk));
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
  // Phi = -A_11^-1 A_1R on the dual slots; by the block inverse of A~ this is
  // G_Gam Kc (the type-1 block of A~^-1 E_R times the coarse Schur complement)
  MatC GK = matmul(GG, C.Kc);
  C.Phi = GK;
  MatC Dc = matmul(GK, transpose(GG));
  for (size_t i = 0; i < Dc.a.size(); ++i) Dc.a[i] = H.a[i] - Dc.a[i];
  C.Op1 = MatC(m + nr, m);
  for (int b = 0; b < m; ++b) {
    for (int a = 0; a < m; ++a) C.Op1(a, b) = Dc(a, b);
    for (int r = 0; r < nr; ++r) C.Op1(m + r, b) = C.Phi(b, r);
  }
  // Laplace-only blocks of the preconditioner (Sec. 2.3.3).  S_b: Schur
  // complement of A~_L onto the side modes (interior eliminated); its block on
  // the dual slots is the Dirichlet block Se, and eliminating the remaining
  // type-1 side modes from it leaves the element's Laplace coarse matrix KL.
  std::vector<int> bmodes, imodes;
  for (int md = 0; md < n2; ++md) {
    int ix = md % n, iy = md / n;
    if (ix >= 2 && iy >= 2) imodes.push_back(md);
    else bmodes.push_back(md);
  }
  auto AL = [&](int a, int b) {
    int i1 = a % n, i2 = a / n, j1 = b % n, j2 = b / n;
    return axx * (C.hy / C.hx) * Mt(i2, j2) * Kt(i1, j1) + ayy * (C.hx / C.hy) * Kt(i2, j2) * Mt(i1, j1);
  };
  int nb = int(bmodes.size()), ni = int(imodes.size());
  MatC Abb(nb, nb), Abi(nb, ni), Aii(ni, ni);
  for (int b = 0; b < nb; ++b)
    for (int a = 0; a < nb; ++a) Abb(a, b) = AL(bmodes[a], bmodes[b]);
  for (int b = 0; b < ni; ++b)
    for (int a = 0; a < nb; ++a) Abi(a, b) = AL(bmodes[a], imodes[b]);
  for (int b = 0; b < ni; ++b)
    for (int a = 0; a < ni; ++a) Aii(a, b) = AL(imodes[a], imodes[b]);
  MatC Sb = Abb;
  if (ni > 0) {
    MatC X = solve(Aii, transpose(Abi));
    MatC AX = matmul(Abi, X);
    for (size_t i = 0; i < Sb.a.size(); ++i) Sb.a[i] -= AX.a[i];
  }
  std::vector<int> bpos(n2, -1), inR(n2, 0);
  for (int a = 0; a < nb; ++a) bpos[bmodes[a]] = a;
  for (int r : C.R) inR[r] = 1;
  C.Se = MatC(m, m);
  for (int b = 0; b < m; ++b)
    for (int a = 0; a < m; ++a) C.Se(a, b) = Sb(bpos[C.Gam[a]], bpos[C.Gam[b]]);
  std::vector<int> e1;
  for (int md : bmodes)
    if (!inR[md]) e1.push_back(md);
  int ne = int(e1.size());
  C.KL = MatC(nr, nr);
  for (int b = 0; b < nr; ++b)
    for (int a = 0; a < nr; ++a) C.KL(a, b) = Sb(bpos[C.R[a]], bpos[C.R[b]]);
  if (ne > 0) {
    MatC S11(ne, ne), S1R(ne, nr);
    for (int b = 0; b < ne; ++b)
      for (int a = 0; a < ne; ++a) S11(a, b) = Sb(bpos[e1[a]], bpos[e1[b]]);
    for (int b = 0; b < nr; ++b)
      for (int a = 0; a < ne; ++a) S1R(a, b) = Sb(bpos[e1[a]], bpos[C.R[b]]);
    MatC X = solve(S11, S1R);
    MatC RX = matmul(transpose(S1R), X);
    for (size_t i = 0; i < C.KL.a.size(); ++i) C.KL.a[i] -= RX.a[i];
  }
}

// Coarse unknown -> coarse modes (transpose of T) and, with c2, the transpose of C_2.
void build_transposes(Handle& h, bool c2) {
  h.cdof_ptr.assign(h.nK + 1, 0);
  for (int d : h.t_dof) h.cdof_ptr[d + 1]++;
  for (int i = 0; i < h.nK; ++i) h.cdof_ptr[i + 1] += h.cdof_ptr[i];
  h.cdof_list.assign(h.t_dof.size(), 0);
  h.cdof_coef.assign(h.t_dof.size(), 0.0);
  {
    std::vector<int> fill(h.cdof_ptr.begin(), h.cdof_ptr.end() - 1);
    for (int i = 0; i < h.ncm; ++i)
      for (int t = h.t_ptr[i]; t < h.t_ptr[i + 1]; ++t) {
        int d = h.t_dof[t], at = fill[d]++;
        h.cdof_list[at] = i;
        h.cdof_coef[at] = h.t_coef[t];
      }
  }
  if (!c2) return;
  h.c2t_ptr.assign(h.nK + 1, 0);
  for (int d : h.c2_dof) h.c2t_ptr[d + 1]++;
  for (int i = 0; i < h.nK; ++i) h.c2t_ptr[i + 1] += h.c2t_ptr[i];
  h.c2t_row.assign(h.c2_dof.size(), 0);
  h.c2t_coef.assign(h.c2_dof.size(), 0.0);
  std::vector<int> fill(h.c2t_ptr.begin(), h.c2t_ptr.end() - 1);
  for (int r = 0; r < h.nlam; ++r)
    for (int t = h.c2_ptr[r]; t < h.c2_ptr[r + 1]; ++t) {
      int at = fill[h.c2_dof[t]]++;
      h.c2t_row[at] = r;
      h.c2t_coef[at] = h.c2_coef[t];
    }
}

// Renumber the coarse unknowns by breadth-first level sets of the coupling
// graph of K (unknowns sharing an element), started from the unknowns of
// smallest y: a level set only couples to its two neighbours, which keeps K
// banded (the order of the dense inverse and of the band-factor byte count).
void order_coarse_levels(Handle& h) {
  const int nK = h.nK, E = h.E;
  std::vector<std::vector<int>> elem_dofs(E);
  for (int e = 0; e < E; ++e) {
    auto& v = elem_dofs[e];
    for (int i = h.cm_off[e]; i < h.cm_off[e + 1]; ++i)
      for (int t = h.t_ptr[i]; t < h.t_ptr[i + 1]; ++t) v.push_back(h.t_dof[t]);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  std::vector<std::vector<int>> dof_elems(nK);
  for (int e = 0; e < E; ++e)
    for (int d : elem_dofs[e]) dof_elems[d].push_back(e);
  std::vector<int> lev(nK, -1), front;
  double ymin = 1e300;
  for (int d = 0; d < nK; ++d) ymin = std::min(ymin, h.dof_y[d]);
  for (int d = 0; d < nK; ++d)
    if (h.dof_y[d] == ymin) { lev[d] = 0; front.push_back(d); }
  std::vector<std::vector<int>> levels{front};
  while (!front.empty()) {
    std::vector<int> next;
    for (int d : front)
      for (int e : dof_elems[d])
        for (int o : elem_dofs[e])
          if (lev[o] < 0) { lev[o] = int(levels.size()); next.push_back(o); }
    if (!next.empty()) levels.push_back(next);
    front.swap(next);
  }
  for (int d = 0; d < nK; ++d)
    if (lev[d] < 0) fail(HDP_E_MESH, "coarse space not connected");
  std::vector<int> perm(nK);   // old -> new
  int pos = 0;
  for (size_t L = 0; L < levels.size(); ++L) {
    std::vector<int> lv = levels[L];
    std::sort(lv.begin(), lv.end());
    for (int d : lv) perm[d] = pos++;
  }
  for (auto& d : h.t_dof) d = perm[d];
  for (auto& d : h.c2_dof) d = perm[d];
  std::vector<double> x(nK), y(nK);
  std::vector<char> vt(nK);
  for (int d = 0; d < nK; ++d) {
    x[perm[d]] = h.dof_x[d];
    y[perm[d]] = h.dof_y[d];
    vt[perm[d]] = h.dof_vtx[d];
  }
  h.dof_x.swap(x);
  h.dof_y.swap(y);
  h.dof_vtx.swap(vt);
  build_transposes(h, true);
}

// Coarse unknowns that share an element (the sparsity of K), as sorted lists.
static std::vector<std::vector<int>> coarse_adjacency(const Handle& h) {
  std::vector<std::vector<int>> elem_dofs(h.E);
  for (int e = 0; e < h.E; ++e) {
    auto& v = elem_dofs[e];
    for (int i = h.cm_off[e]; i < h.cm_off[e + 1]; ++i)
      for (int t = h.t_ptr[i]; t < h.t_ptr[i + 1]; ++t) v.push_back(h.t_dof[t]);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  std::vector<std::vector<int>> adj(h.nK);
  for (int e = 0; e < h.E; ++e)
    for (int a : elem_dofs[e])
      for (int b : elem_dofs[e])
        if (a != b) adj[a].push_back(b);
  for (auto& v : adj) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  return adj;
}

// Nested-dissection order of the coarse unknowns for the multifrontal coarse
// factor (recursive coordinate bisection).  A set is cut at the line through
// a column (or row) of mesh vertices near its median, across its longer
// extent; the unknowns on the far side that share an element with the near
// side form the separator, so the two remaining parts share no element and are
// eliminated independently.  Sets of at most `leaf` unknowns are leaves.
// Nodes are numbered in postorder (children before parents); the unknowns a
// node owns are consecutive in the new numbering, and its boundary lists the
// later (ancestor) unknowns its subtree is coupled to after elimination.
void order_coarse_nd(Handle& h, size_t leaf) {
  const int nK = h.nK;
  const auto adj = coarse_adjacency(h);
  struct Node { std::vector<int> own; int child[2] = {-1, -1}; int depth = 0; };
  std::vector<Node> nodes;
  std::vector<int> side(nK, -1);
  std::function<int(std::vector<int>&, int)> build = [&](std::vector<int>& S, int depth) -> int {
    const int id = int(nodes.size());
    nodes.emplace_back();
    nodes[id].depth = depth;
    if (S.size() <= leaf) {
      nodes[id].own = S;
      return id;
    }
    double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
    for (int u : S) {
      lo[0] = std::min(lo[0], h.dof_x[u]); hi[0] = std::max(hi[0], h.dof_x[u]);
      lo[1] = std::min(lo[1], h.dof_y[u]); hi[1] = std::max(hi[1], h.dof_y[u]);
    }
    std::vector<int> best_sep, best_a, best_b;
    double best_score = 1e300;
    for (int axis : {hi[0] - lo[0] >= hi[1] - lo[1] ? 0 : 1, hi[0] - lo[0] >= hi[1] - lo[1] ? 1 : 0}) {
      const std::vector<double>& c = axis == 0 ? h.dof_x : h.dof_y;
      std::vector<double> cs;
      for (int u : S) cs.push_back(c[u]);
      std::sort(cs.begin(), cs.end());
      std::vector<double> lines;   // vertex coordinates present in the set
      for (int u : S)
        if (h.dof_vtx[u]) lines.push_back(c[u]);
      std::sort(lines.begin(), lines.end());
      lines.erase(std::unique(lines.begin(), lines.end()), lines.end());
      if (lines.empty()) continue;
      // the vertex lines nearest to the median of the set, a few on each side
      const double med = cs[cs.size() / 2];
      const size_t at = size_t(std::lower_bound(lines.begin(), lines.end(), med) - lines.begin());
      for (size_t q = at >= 3 ? at - 3 : 0; q < std::min(lines.size(), at + 4); ++q) {
        const double m = lines[q];
        for (int u : S) side[u] = c[u] < m ? 0 : 1;
        std::vector<int> sep, a, b;
        for (int u : S) {
          if (side[u] == 0) { a.push_back(u); continue; }
          bool touch = false;
          for (int v : adj[u])
            if (side[v] == 0) { touch = true; break; }
          (touch ? sep : b).push_back(u);
        }
        for (int u : S) side[u] = -1;
        if (a.empty() || b.empty()) continue;
        const double imb = std::abs(double(a.size()) - double(b.size())) / double(S.size());
        const double score = double(sep.size()) * (1.0 + 2.0 * imb);
        if (score < best_score) {
          best_score = score;
          best_sep.swap(sep); best_a.swap(a); best_b.swap(b);
        }
      }
      if (best_score < 1e300) break;   // the longer extent gave a cut
    }
    if (best_score >= 1e300 || best_sep.size() * 2 > S.size()) {
      nodes[id].own = S;   // no useful cut: one dense node
      return id;
    }
    S.clear();
    S.shrink_to_fit();
    nodes[id].own = best_sep;
    const int ca = build(best_a, depth + 1);
    const int cb = build(best_b, depth + 1);
    nodes[id].child[0] = ca;
    nodes[id].child[1] = cb;
    return id;
  };
  std::vector<int> all(nK);
  for (int u = 0; u < nK; ++u) all[u] = u;
  const int root = build(all, 0);
  // postorder numbering of nodes and unknowns
  std::vector<int> post;   // node ids in postorder
  std::function<void(int)> walk = [&](int t) {
    for (int c : nodes[t].child)
      if (c >= 0) walk(c);
    post.push_back(t);
  };
  walk(root);
  const int nn = int(post.size());
  std::vector<int> pos_of(nodes.size());
  for (int q = 0; q < nn; ++q) pos_of[post[q]] = q;
  std::vector<int> perm(nK, -1);   // old -> new
  h.nd_off.assign(nn + 1, 0);
  h.nd_depth.assign(nn, 0);
  h.nd_child.assign(2 * size_t(nn), -1);
  int at = 0;
  for (int q = 0; q < nn; ++q) {
    const Node& N = nodes[post[q]];
    std::vector<int> own = N.own;
    std::sort(own.begin(), own.end());
    for (int u : own) perm[u] = at++;
    h.nd_off[q + 1] = at;
    h.nd_depth[q] = N.depth;
    for (int k = 0; k < 2; ++k) h.nd_child[2 * size_t(q) + k] = N.child[k] >= 0 ? pos_of[N.child[k]] : -1;
  }
  if (at != nK) fail(HDP_E_MESH, "nested dissection lost coarse unknowns");
  // boundaries: own neighbours and children's boundaries beyond the node's range
  std::vector<std::vector<int>> bnd(nn);
  for (int q = 0; q < nn; ++q) {
    const int end = h.nd_off[q + 1];
    std::vector<int> b;
    for (int u : nodes[post[q]].own)
      for (int v : adj[u])
        if (perm[v] >= end) b.push_back(perm[v]);
    for (int k = 0; k < 2; ++k) {
      const int c = h.nd_child[2 * size_t(q) + k];
      if (c < 0) continue;
      for (int v : bnd[c])
        if (v >= end) b.push_back(v);
    }
    std::sort(b.begin(), b.end());
    b.erase(std::unique(b.begin(), b.end()), b.end());
    bnd[q].swap(b);
  }
  h.nd_boff.assign(nn + 1, 0);
  h.nd_bnd.clear();
  for (int q = 0; q < nn; ++q) {
    h.nd_bnd.insert(h.nd_bnd.end(), bnd[q].begin(), bnd[q].end());
    h.nd_boff[q + 1] = int64_t(h.nd_bnd.size());
  }
  for (auto& d : h.t_dof) d = perm[d];
  for (auto& d : h.c2_dof) d = perm[d];
  std::vector<double> x(nK), y(nK);
  std::vector<char> vt(nK);
  for (int d = 0; d < nK; ++d) {
    x[perm[d]] = h.dof_x[d];
    y[perm[d]] = h.dof_y[d];
    vt[perm[d]] = h.dof_vtx[d];
  }
  h.dof_x.swap(x);
  h.dof_y.swap(y);
  h.dof_vtx.swap(vt);
  build_transposes(h, true);
}

// Preconditioner blocks on the dual rows that C_2 touches (hanging edges).
// The literal nullspace basis of Sec. 2.3.2 projects each kept unknown onto
// null(C_p) orthogonally; in terms of the expansions T used here (kept
// unknown = coarse unknown, T_2 = the type-2 part of the basis) that basis is
// Z_2 = T_2 G^-1 with the Gram matrix G = T_2^T T_2.  So C_2 = C_2^T G^-1 and
// the Laplace coarse matrix is G^-1 KL G^-1, and the terms C_2 C_2^T of
// C W C^T and C_2 KL C_2^T of the preconditioner (Sec. 2.3.3) become dense
// blocks over the hanging rows of each connected group of coarse unknowns.
void build_hanging_blocks(Handle& h) {
  const int nlam = h.nlam, nK = h.nK;
  std::vector<char> is_h(nlam, 0);
  h.row_xinv.assign(nlam, 0.0);
  std::vector<double> D(nlam, 0.0);
  for (int r = 0; r < nlam; ++r) {
    is_h[r] = h.c2_ptr[r + 1] > h.c2_ptr[r];
    D[r] = h.row_coef[2 * r] * h.row_coef[2 * r] + h.row_coef[2 * r + 1] * h.row_coef[2 * r + 1];
    if (is_h[r]) h.row_xinv[r] = 1.0;
    else if (D[r] > 0) h.row_xinv[r] = 1.0 / D[r];
    else fail(HDP_E_MESH, "dual row without entries");
  }
  h.hb_off.assign(1, 0);
  h.hb_rows.clear();
  h.hb_moff.assign(1, 0);
  h.hb_xinv.clear();
  h.hb_y2.clear();
  h.nh = 0;
  // groups: coarse unknowns that share a coarse-mode expansion or a C_2 row
  std::vector<int> par(nK);
  for (int i = 0; i < nK; ++i) par[i] = i;
  std::function<int(int)> find = [&](int x) { return par[x] == x ? x : par[x] = find(par[x]); };
  auto unite = [&](int a, int b) { a = find(a); b = find(b); if (a != b) par[a] = b; };
  for (int i = 0; i < h.ncm; ++i)
    for (int t = h.t_ptr[i] + 1; t < h.t_ptr[i + 1]; ++t) unite(h.t_dof[h.t_ptr[i]], h.t_dof[t]);
  for (int r = 0; r < nlam; ++r)
    for (int t = h.c2_ptr[r] + 1; t < h.c2_ptr[r + 1]; ++t) unite(h.c2_dof[h.c2_ptr[r]], h.c2_dof[t]);
  std::map<int, std::vector<int>> grp_rows;
  for (int r = 0; r < nlam; ++r)
    if (is_h[r]) grp_rows[find(h.c2_dof[h.c2_ptr[r]])].push_back(r);
  if (grp_rows.empty()) return;
  std::map<int, std::vector<int>> grp_dofs;
  for (int d = 0; d < nK; ++d) {
    int g = find(d);
    if (grp_rows.count(g)) grp_dofs[g].push_back(d);
  }
  // element of each coarse mode
  std::vector<int> cm_elem(h.ncm);
  for (int e = 0; e < h.E; ++e)
    for (int i = h.cm_off[e]; i < h.cm_off[e + 1]; ++i) cm_elem[i] = e;
  for (auto& gr : grp_rows) {
    const std::vector<int>& rows = gr.second;
    const std::vector<int>& S = grp_dofs[gr.first];
    int ns = int(S.size()), nr = int(rows.size());
    std::map<int, int> pos;
    for (int a = 0; a < ns; ++a) pos[S[a]] = a;
    // Gram matrix and Laplace coarse matrix restricted to the group
    MatD G(ns, ns), KL(ns, ns);
    std::set<int> elems;
    for (int d : S)
      for (int t = h.cdof_ptr[d]; t < h.cdof_ptr[d + 1]; ++t) elems.insert(cm_elem[h.cdof_list[t]]);
    for (int e : elems) {
      const ElemClass& C = h.classes[h.cls[e]];
      int co = h.cm_off[e];
      for (int a = 0; a < C.nr; ++a) {
        int ia = co + a;
        bool in_a = pos.count(h.t_dof[h.t_ptr[ia]]) > 0;
        if (in_a)
          for (int t = h.t_ptr[ia]; t < h.t_ptr[ia + 1]; ++t)
            for (int u = h.t_ptr[ia]; u < h.t_ptr[ia + 1]; ++u)
              G(pos[h.t_dof[t]], pos[h.t_dof[u]]) += h.t_coef[t] * h.t_coef[u];
        if (!in_a) continue;
        for (int b = 0; b < C.nr; ++b) {
          int ib = co + b;
          if (!pos.count(h.t_dof[h.t_ptr[ib]])) continue;
          double kab = C.KL(a, b).real();   // real: layers are refused with hanging edges
          for (int t = h.t_ptr[ia]; t < h.t_ptr[ia + 1]; ++t)
            for (int u = h.t_ptr[ib]; u < h.t_ptr[ib + 1]; ++u)
              KL(pos[h.t_dof[t]], pos[h.t_dof[u]]) += h.t_coef[t] * kab * h.t_coef[u];
        }
      }
    }
    MatD Gi = inverse(G);
    MatD C2(nr, ns);
    for (int i = 0; i < nr; ++i)
      for (int t = h.c2_ptr[rows[i]]; t < h.c2_ptr[rows[i] + 1]; ++t) C2(i, pos[h.c2_dof[t]]) += h.c2_coef[t];
    MatD M = matmul(C2, Gi);
    MatD X = matmul(M, transpose(M));
    for (int i = 0; i < nr; ++i) X(i, i) += D[rows[i]];
    MatD Y2 = matmul(matmul(M, matmul(matmul(Gi, KL), Gi)), transpose(M));
    MatD Xi = inverse(X);
    h.hb_rows.insert(h.hb_rows.end(), rows.begin(), rows.end());
    h.hb_off.push_back(int(h.hb_rows.size()));
    h.hb_xinv.insert(h.hb_xinv.end(), Xi.a.begin(), Xi.a.end());
    h.hb_y2.insert(h.hb_y2.end(), Y2.a.begin(), Y2.a.end());
    h.hb_moff.push_back(int64_t(h.hb_xinv.size()));
  }
  h.nh = int(h.hb_rows.size());
}

}  // namespace

void coarse_coo(const Handle& h, std::vector<int64_t>& kidx, std::vector<double2>& kval) {
  std::vector<std::pair<int64_t, cd>> coo;
  for (int e = 0; e < h.E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    const int co = h.cm_off[e];
    for (int b = 0; b < C.nr; ++b)
      for (int a = 0; a < C.nr; ++a) {
        cd kab = C.Kc(a, b);
        for (int t = h.t_ptr[co + a]; t < h.t_ptr[co + a + 1]; ++t)
          for (int u = h.t_ptr[co + b]; u < h.t_ptr[co + b + 1]; ++u)
            coo.push_back({h.t_dof[t] + int64_t(h.nK) * h.t_dof[u], h.t_coef[t] * kab * h.t_coef[u]});
      }
  }
  std::sort(coo.begin(), coo.end(), [](auto& x, auto& y) { return x.first < y.first; });
  kidx.clear();
  kval.clear();
  for (size_t t = 0; t < coo.size();) {
    int64_t key = coo[t].first;
    cd s = 0;
    while (t < coo.size() && coo[t].first == key) s += coo[t++].second;
    kidx.push_back(key);
    kval.push_back(make_double2(s.real(), s.imag()));
  }
}

// Bytes of a banded (envelope) LU factor of K in its natural order: row i of L
// spans columns first_i..i, and U mirrors it (K is structurally symmetric); what
// one coarse solve with such a factor reads.  kidx: sorted COO keys row + nK col.
double coarse_band_bytes(int nK, const std::vector<int64_t>& kidx) {
  std::vector<int> first(static_cast<size_t>(nK));
  for (int i = 0; i < nK; ++i) first[size_t(i)] = i;
  for (int64_t key : kidx) {
    const int64_t r = key % nK, c = key / nK;
    first[size_t(r)] = std::min(first[size_t(r)], int(c));
  }
  double env = 0;
  for (int i = 0; i < nK; ++i) env += double(i - first[size_t(i)] + 1);
  return 16.0 * (2.0 * env - double(nK));
}

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
  h.sigx.assign(E, 0.0);
  h.sigy.assign(E, 0.0);
  h.pml = false;
  if (prob->pml_sigma)
    for (int e = 0; e < E; ++e) {
      const double a = prob->pml_sigma[2 * e], b = prob->pml_sigma[2 * e + 1];
      if (!std::isfinite(a) || !std::isfinite(b) || a < 0 || b < 0) fail(HDP_E_ARG, "pml_sigma not finite or negative");
      h.sigx[e] = a;
      h.sigy[e] = b;
      if (a != 0 || b != 0) h.pml = true;
    }
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
  // sides: neighbours along the same grid line.  A side either matches one
  // neighbour side exactly (conforming), lies inside one longer neighbour side
  // (fine side of a hanging edge) or holds several shorter ones (coarse side).
  struct Seg { int64_t lo, hi; int e, s; };
  std::map<std::pair<int, int64_t>, std::vector<Seg>> facing[2];   // [0]: sides 1,3; [1]: sides 2,4
  auto key_of = [&](int e, int s) {
    switch (s) {
      case 1: return SideKey{0, X0[e], Y0[e], Y1[e]};
      case 2: return SideKey{0, X1[e], Y0[e], Y1[e]};
      case 3: return SideKey{1, Y0[e], X0[e], X1[e]};
      default: return SideKey{1, Y1[e], X0[e], X1[e]};
    }
  };
  for (int e = 0; e < E; ++e)
    for (int s = 1; s <= 4; ++s) {
      SideKey k = key_of(e, s);
      facing[(s - 1) % 2][{k.kind, k.c}].push_back({k.lo, k.hi, e, s});
    }
  h.side_type.assign(4 * E, 0);
  h.side_le.assign(4 * E, 0);
  h.nb_e.assign(4 * E, -1);
  h.nb_s.assign(4 * E, 0);
  h.side_a.assign(4 * E, 1.0);
  h.side_b.assign(4 * E, 0.0);
  h.side_nbrs.assign(4 * E, {});
  h.bmask.assign(E, 0);
  for (int e = 0; e < E; ++e)
    for (int s = 1; s <= 4; ++s) {
      const int si = 4 * e + s - 1;
      SideKey key = key_of(e, s);
      bool bnd = (key.kind == 0 && (key.c == 0 || key.c == NX)) ||
                 (key.kind == 1 && (key.c == 0 || key.c == NY));
      if (bnd) { h.bmask[e] |= 1 << (s - 1); continue; }
      std::vector<Seg> ov;
      for (const Seg& o : facing[s % 2][{key.kind, key.c}])
        if (std::min(o.hi, key.hi) > std::max(o.lo, key.lo)) ov.push_back(o);
      if (ov.empty()) fail(HDP_E_MESH, "interior side without a neighbour");
      if (ov.size() == 1 && ov[0].lo == key.lo && ov[0].hi == key.hi) {
        h.side_type[si] = 1;
        h.nb_e[si] = ov[0].e;
        h.nb_s[si] = ov[0].s;
      } else if (ov.size() == 1 && ov[0].lo <= key.lo && ov[0].hi >= key.hi) {
        h.side_type[si] = 2;
        h.nb_e[si] = ov[0].e;
        h.nb_s[si] = ov[0].s;
        double L = double(ov[0].hi - ov[0].lo);
        h.side_a[si] = double(key.hi - key.lo) / L;
        h.side_b[si] = double(key.lo + key.hi - ov[0].lo - ov[0].hi) / L;
      } else {
        int64_t covered = 0;
        for (const Seg& o : ov) {
          if (o.lo < key.lo || o.hi > key.hi) fail(HDP_E_MESH, "overlapping leaves");
          covered += o.hi - o.lo;
          h.side_nbrs[si].push_back(o.e);
        }
        if (covered != key.hi - key.lo) fail(HDP_E_MESH, "side not covered by its neighbours");
        h.side_type[si] = 3;
      }
      if (h.side_type[si] != 1) h.nonconforming = true;
    }
  // coarse order l (Sec. 2.3.4): the criterion is evaluated for every element with
  // its longest edge and its local wavenumber k sqrt(eps_r), and the largest value
  // is used (with eps_r = 1 this is the free-space k and the longest edge); with
  // l_free_space the free-space k everywhere (the longest edge of the mesh, as in
  // the paper's dielectric-cylinder example)
  const bool free_k = prob->l_free_space != 0;
  auto k_of = [&](int f) { return free_k ? prob->k : prob->k * std::sqrt(std::max(h.eps[f], 0.0)); };
  double khmax = 0;
  for (int e = 0; e < E; ++e) khmax = std::max(khmax, k_of(e) * std::max(h.hx[e], h.hy[e]));
  h.l = prob->l > 0 ? prob->l : dispersion_l(khmax, 1.0) + std::max(0, prob->l_safety);
  // per-edge orders (l_per_edge): the rule on each edge with, for every leaf
  // touching it, its own side length along the edge and k sqrt(eps_r); a fine
  // side of a hanging edge takes the value of the coarse side that holds it
  std::vector<int> l_side(4 * size_t(E), h.l);
  if (prob->l <= 0 && prob->l_per_edge) {
    auto len = [&](int f, int s) { return s <= 2 ? h.hy[f] : h.hx[f]; };
    auto rule = [&](int f, int s) {
      return dispersion_l(k_of(f) * len(f, s), 1.0);
    };
    int lmax = 1;
    for (int e = 0; e < E; ++e)
      for (int s = 1; s <= 4; ++s) {
        int ee = e, ss = s;
        if (h.side_type[4 * e + s - 1] == 2) { ee = h.nb_e[4 * e + s - 1]; ss = h.nb_s[4 * e + s - 1]; }
        const int sj = 4 * ee + ss - 1;
        int v = rule(ee, ss);
        if (h.side_type[sj] == 1) v = std::max(v, rule(h.nb_e[sj], h.nb_s[sj]));
        if (h.side_type[sj] == 3)
          for (int f : h.side_nbrs[sj]) v = std::max(v, rule(f, ss % 2 == 1 ? ss + 1 : ss - 1));
        v += std::max(0, prob->l_safety);
        l_side[4 * e + s - 1] = v;
        lmax = std::max(lmax, v);
      }
    h.l = lmax;
  }
  // per side: the primal count le = min(l, p, p_neighbour) of its edge and the
  // highest bubble index among the element's coarse modes
  // and the highest dual-slot bubble gtop: p, or on the fine side of a hanging
  // edge the last degree whose constraint diagonal a^k stays above discard_tol
  const double tau = std::max(0.0, prob->discard_tol);
  if (!std::isfinite(prob->discard_tol)) fail(HDP_E_ARG, "discard_tol not finite");
  h.discard_tol = tau;
  std::vector<std::array<int, 8>> tops(E);
  for (int e = 0; e < E; ++e)
    for (int s = 1; s <= 4; ++s) {
      const int si = 4 * e + s - 1, p = h.deg[e];
      int le = std::min(l_side[si], p), top = le, gtop = p;
      if (h.side_type[si] == 1 || h.side_type[si] == 2) le = top = std::min(le, h.deg[h.nb_e[si]]);
      else if (h.side_type[si] == 3) top = p;
      if (h.side_type[si] == 0) gtop = top;
      if (h.side_type[si] == 2)
        while (gtop > le && std::pow(h.side_a[si], gtop) < tau) --gtop;
      h.side_le[si] = le;
      tops[e][s - 1] = top;
      tops[e][4 + s - 1] = gtop;
    }
  // Robin-modified local problems (Sec. 2.3.4): labels from the levels of a
  // breadth-first spanning tree of the element adjacency; the term goes on an
  // interior side when every neighbour across it has the opposite label
  h.rmask.assign(E, 0);
  if (prob->robin_modified) {
    auto nbrs = [&](int e, int s) {
      const int si = 4 * e + s - 1;
      std::vector<int> v;
      if (h.side_type[si] == 1 || h.side_type[si] == 2) v.push_back(h.nb_e[si]);
      else if (h.side_type[si] == 3) v = h.side_nbrs[si];
      std::sort(v.begin(), v.end());
      return v;
    };
    std::vector<int> depth(E, -1);
    std::vector<int> queue{0};
    depth[0] = 0;
    for (size_t q = 0; q < queue.size(); ++q) {
      const int e = queue[q];
      for (int s = 1; s <= 4; ++s)
        for (int f : nbrs(e, s))
          if (depth[f] < 0) {
            depth[f] = depth[e] + 1;
            queue.push_back(f);
          }
    }
    for (int e = 0; e < E; ++e)
      if (depth[e] < 0) fail(HDP_E_MESH, "mesh is not connected");
    for (int e = 0; e < E; ++e)
      for (int s = 1; s <= 4; ++s) {
        const std::vector<int> v = nbrs(e, s);
        if (v.empty()) continue;
        int opp = 0;
        for (int f : v) opp += (depth[f] % 2) != (depth[e] % 2);
        if (opp == 0) continue;
        if (opp != int(v.size()))
          fail(HDP_E_UNSUPPORTED, "Robin-modified local problems: side " + std::to_string(s) + " of leaf " +
                                      std::to_string(e) + " has neighbours of both labels");
        h.rmask[e] |= (depth[e] % 2 == 0 ? 2 : 1) << (2 * (s - 1));
      }
  }
  if (h.pml && h.nonconforming)
    fail(HDP_E_UNSUPPORTED, "perfectly matched layers on a mesh with hanging edges");
  // classes
  std::map<std::tuple<int, double, double, double, int, int, std::array<int, 8>, std::pair<double, double>>, int>
      cmap;
  h.cls.resize(E);
  for (int e = 0; e < E; ++e) {
    auto key = std::make_tuple(h.deg[e], h.hx[e], h.hy[e], h.eps[e], h.bmask[e], h.rmask[e], tops[e],
                               std::make_pair(h.sigx[e], h.sigy[e]));
    auto it = cmap.find(key);
    if (it == cmap.end()) {
      ElemClass C;
      C.p = h.deg[e]; C.n = C.p + 1; C.hx = h.hx[e]; C.hy = h.hy[e];
      C.eps = h.eps[e]; C.bmask = h.bmask[e]; C.rmask = h.rmask[e];
      C.sigx = h.sigx[e]; C.sigy = h.sigy[e];
      for (int s = 0; s < 4; ++s) {
        C.top[s] = tops[e][s];
        C.gtop[s] = tops[e][4 + s];
      }
      it = cmap.emplace(key, int(h.classes.size())).first;
      h.classes.push_back(C);
    }
    h.cls[e] = it->second;
    h.classes[it->second].elems.push_back(e);
  }
  // classes are independent: build them on host threads (an error in any
  // class is rethrown after all threads have joined)
  {
    const auto tc = std::chrono::steady_clock::now();
    const int nthreads = int(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    std::atomic<int> next{0};
    std::exception_ptr err;
    std::mutex err_mu;
    auto work = [&] {
      for (int c = next++; c < int(h.classes.size()); c = next++) {
        try {
          build_class(h.classes[c], h.k);
        } catch (...) {
          std::lock_guard<std::mutex> lock(err_mu);
          if (!err) err = std::current_exception();
        }
      }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < std::min<int>(nthreads, int(h.classes.size())); ++t) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    if (err) std::rethrow_exception(err);
    h.setup_classes_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tc).count();
  }
  h.min_margin = 1;
  for (auto& C : h.classes) h.min_margin = std::min(h.min_margin, C.margin);
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
    for (int t = 1; t < s; ++t) pos += C.gtop[t - 1] - C.top[t - 1];
    return h.slot_off[e] + pos + (kk - C.top[s - 1] - 1);
  };
  // ---- coarse unknowns and the coarse-mode expansions T ----------------------
  // Geometric points on the finest grid.  A point strictly inside a side is a
  // hanging point: its value is the trace of that (coarse) side there.
  using Pt = std::pair<int64_t, int64_t>;
  std::map<Pt, std::pair<int, int>> owner;   // hanging point -> (element, side) holding it
  for (int e = 0; e < E; ++e)
    for (int s = 1; s <= 4; ++s) {
      const int si = 4 * e + s - 1;
      if (h.side_type[si] != 3) continue;
      SideKey k = key_of(e, s);
      for (int f : h.side_nbrs[si]) {
        int64_t ends[2] = {k.kind == 0 ? Y0[f] : X0[f], k.kind == 0 ? Y1[f] : X1[f]};
        for (int64_t q : ends)
          if (q > k.lo && q < k.hi) owner[k.kind == 0 ? Pt{k.c, q} : Pt{q, k.c}] = {e, s};
      }
    }
  std::map<std::tuple<int, int64_t, int64_t, int64_t, int>, int> cids;
  auto dof_id = [&](const std::tuple<int, int64_t, int64_t, int64_t, int>& key) {
    auto it = cids.find(key);
    if (it == cids.end()) it = cids.emplace(key, int(cids.size())).first;
    return it->second;
  };
  auto bubble_dof = [&](int e, int s, int kk) {
    SideKey sk = key_of(e, s);
    return dof_id(std::make_tuple(sk.kind, sk.c, sk.lo, sk.hi, kk));
  };
  // corner (ix, iy) of element e: ix = 0 right, 1 left; iy = 0 top, 1 bottom
  auto corner = [&](int e, int ix, int iy) { return Pt{ix == 0 ? X1[e] : X0[e], iy == 0 ? Y1[e] : Y0[e]}; };
  // end of side s at parameter +1 / -1 (parameter along increasing x or y)
  auto side_end = [&](int e, int s, bool plus) {
    if (s <= 2) return corner(e, s == 2 ? 0 : 1, plus ? 0 : 1);
    return corner(e, plus ? 0 : 1, s == 4 ? 0 : 1);
  };
  using Expansion = std::map<int, double>;
  std::map<Pt, Expansion> memo;
  std::function<Expansion(const Pt&)> expand = [&](const Pt& P) -> Expansion {
    auto m = memo.find(P);
    if (m != memo.end()) return m->second;
    Expansion out;
    auto o = owner.find(P);
    if (o == owner.end()) {
      out[dof_id(std::make_tuple(-1, P.first, P.second, int64_t(0), 0))] = 1.0;
    } else {
      int c = o->second.first, s = o->second.second;
      SideKey k = key_of(c, s);
      int64_t q = k.kind == 0 ? P.second : P.first;
      double t = 2.0 * double(q - k.lo) / double(k.hi - k.lo) - 1.0;
      int nc = h.deg[c] + 1;
      std::vector<double> v(nc);
      vertex_basis(nc, t, v.data());
      for (auto& kv : expand(side_end(c, s, true))) out[kv.first] += v[0] * kv.second;
      for (auto& kv : expand(side_end(c, s, false))) out[kv.first] += v[1] * kv.second;
      for (int j = 2; j < nc; ++j) out[bubble_dof(c, s, j)] += v[j];
    }
    memo[P] = out;
    return out;
  };
  // restriction of the coarse side's bubbles to a fine side: rho[k][j] is the
  // fine vertex-basis coefficient k of N_j(a s + b) (exact polynomial
  // interpolation at the Gauss-Lobatto nodes of the coarse degree)
  auto restriction = [&](int e, int s) {
    const int si = 4 * e + s - 1;
    int c = h.nb_e[si];
    int nc = h.deg[c] + 1;
    double a = h.side_a[si], b = h.side_b[si];
    std::vector<double> t = gll_nodes(nc), row(nc);
    MatD V(nc, nc), Rh(nc, nc);
    for (int i = 0; i < nc; ++i) {
      vertex_basis(nc, t[i], row.data());
      for (int m = 0; m < nc; ++m) V(i, m) = row[m];
      vertex_basis(nc, a * t[i] + b, row.data());
      for (int j = 0; j < nc; ++j) Rh(i, j) = row[j];
    }
    return solve(V, Rh);   // (nc x nc): [k][j]
  };
  std::map<int, MatD> rho;   // per fine side index si
  for (int e = 0; e < E; ++e)
    for (int s = 1; s <= 4; ++s)
      if (h.side_type[4 * e + s - 1] == 2) rho[4 * e + s - 1] = restriction(e, s);
  h.t_ptr.assign(h.ncm + 1, 0);
  h.t_dof.clear();
  h.t_coef.clear();
  h.cm_mode.assign(h.ncm, 0);
  for (int e = 0; e < E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    for (int r = 0; r < C.nr; ++r) {
      int md = C.R[r], n = C.n, ix = md % n, iy = md / n;
      Expansion ex;
      if (ix < 2 && iy < 2) {
        ex = expand(corner(e, ix, iy));
      } else {
        int s, kk;
        if (ix == 0) { s = 2; kk = iy; }
        else if (ix == 1) { s = 1; kk = iy; }
        else if (iy == 0) { s = 4; kk = ix; }
        else { s = 3; kk = ix; }
        const int si = 4 * e + s - 1;
        if (h.side_type[si] == 2) {
          // fine side of a hanging edge: bubble kk of the restricted coarse trace
          const MatD& rh = rho.at(si);
          int c = h.nb_e[si], sc = h.nb_s[si];
          for (int j = kk; j <= h.deg[c]; ++j) ex[bubble_dof(c, sc, j)] += rh(kk, j);
        } else if (h.side_type[si] == 1) {
          // shared edge: both elements name it by the same segment
          ex[bubble_dof(e, s, kk)] = 1.0;
        } else {
          ex[bubble_dof(e, s, kk)] = 1.0;
        }
      }
      int i = h.cm_off[e] + r;
      h.cm_mode[i] = md;
      for (auto& kv : ex)
        if (kv.second != 0.0) {
          h.t_dof.push_back(kv.first);
          h.t_coef.push_back(kv.second);
        }
      h.t_ptr[i + 1] = int(h.t_dof.size());
    }
  }
  h.nK = int(cids.size());
  // position of each coarse unknown across the mesh (vertex, or edge midpoint) in
  // fine-grid units: orders the coarse unknowns into strips for the coarse factor
  h.dof_y.assign(h.nK, 0.0);
  h.dof_x.assign(h.nK, 0.0);
  h.dof_vtx.assign(h.nK, 0);
  for (auto& kv : cids) {
    const auto& key = kv.first;
    int kind = std::get<0>(key);   // -1 vertex (x, y); 0 side x = c, y in [lo, hi]; 1 side y = c
    double y = kind == -1 ? double(std::get<2>(key))
               : kind == 0 ? 0.5 * double(std::get<2>(key) + std::get<3>(key))
                           : double(std::get<1>(key));
    double x = kind == 1 ? 0.5 * double(std::get<2>(key) + std::get<3>(key)) : double(std::get<1>(key));
    h.dof_y[kv.second] = y;
    h.dof_x[kv.second] = x;
    h.dof_vtx[kv.second] = kind == -1;
  }
  build_transposes(h, false);
  // ---- dual rows in Algorithm 1 visiting order -----------------------------
  std::vector<int> vorder(E);
  for (int e = 0; e < E; ++e) vorder[e] = e;
  std::stable_sort(vorder.begin(), vorder.end(), [&](int a, int b) { return level[a] > level[b]; });
  std::vector<char> visited(4 * E, 0);
  std::map<std::pair<int, int>, std::set<int>> zeroed;   // coarse side -> rows already imposed
  h.row_slot.clear(); h.row_coef.clear();
  h.c2_ptr.assign(1, 0); h.c2_dof.clear(); h.c2_coef.clear();
  h.slot_row.assign(h.nslots, -1);
  h.slot_coef.assign(h.nslots, 0.0);
  h.slot_mode.assign(h.nslots, 0);
  auto add_row = [&](int a, double ca, int b, double cb) {
    int row = int(h.row_coef.size() / 2);
    h.row_slot.push_back(a);
    h.row_coef.push_back(a >= 0 ? ca : 0.0);
    h.row_slot.push_back(b);
    h.row_coef.push_back(b >= 0 ? cb : 0.0);
    if (a >= 0) { h.slot_row[a] = row; h.slot_coef[a] = ca; }
    if (b >= 0) { h.slot_row[b] = row; h.slot_coef[b] = cb; }
    return row;
  };
  for (int e : vorder)
    for (int s = 1; s <= 4; ++s) {
      const int si = 4 * e + s - 1;
      const int type = h.side_type[si];
      if (type == 0 || visited[si]) continue;
      visited[si] = 1;
      if (type == 3) continue;   // imposed from the finer sides
      int c = h.nb_e[si], sc = h.nb_s[si];
      int le = h.side_le[si];
      int L = std::max(h.deg[e], h.deg[c]);
      if (type == 1) {
        visited[4 * c + sc - 1] = 1;
        for (int kk = le + 1; kk <= L; ++kk) {
          add_row(kk <= h.deg[c] ? slot_of(c, sc, kk) : -1, SQ2, kk <= h.deg[e] ? slot_of(e, s, kk) : -1, -SQ2);
          h.c2_ptr.push_back(int(h.c2_dof.size()));
        }
      } else {
        // fine side: [restricted coarse trace]_k - [fine trace]_k; rows whose
        // fine mode does not exist only involve the coarse side and are kept
        // once per coarse side (degree-reduction redundancy)
        const MatD& rh = rho.at(si);
        auto& zs = zeroed[{c, sc}];
        for (int kk = le + 1; kk <= L; ++kk) {
          if (std::pow(h.side_a[si], kk) < tau) break;   // decayed constraint diagonal (Sec. 2.2.4)
          if (kk > h.deg[e]) {
            if (zs.count(kk)) continue;
            zs.insert(kk);
          }
          add_row(-1, 0.0, kk <= h.deg[e] ? slot_of(e, s, kk) : -1, -SQ2);
          for (int j = kk; j <= h.deg[c]; ++j) {
            h.c2_dof.push_back(bubble_dof(c, sc, j));
            h.c2_coef.push_back(SQ2 * rh(kk, j));
          }
          h.c2_ptr.push_back(int(h.c2_dof.size()));
        }
      }
    }
  h.nlam = int(h.row_coef.size() / 2);
  if (int(cids.size()) != h.nK) fail(HDP_E_MESH, "coarse unknown without a coarse mode");
  for (int e = 0; e < E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    for (int g = 0; g < C.m; ++g) {
      h.slot_mode[h.slot_off[e] + g] = C.Gam[g];
      if (h.slot_row[h.slot_off[e] + g] < 0) fail(HDP_E_MESH, "dual slot without a row");
    }
  }
  build_transposes(h, true);
  build_hanging_blocks(h);
  // coarse factor: dense inverse for small coarse spaces (one streaming GEMV per
  // solve, 164 MB at 3,201 unknowns), the nested-dissection factor beyond 6,000
  // (a requested factor gets small blocks, so that small meshes exercise it too;
  // solves of 9 or more columns take leaves of up to 192 unknowns, whose fewer,
  // fuller launches are faster there: 0.476 against 0.483 ms per 64-column solve
  // on the 64x64 scatterer, where one column keeps 96)
  const bool requested = h.coarse_mode >= 0;
  if (h.coarse_mode < 0) h.coarse_mode = h.nK > 6000 ? 2 : 0;
  if (h.coarse_mode == 2) order_coarse_nd(h, requested ? 32 : (h.max_rhs >= 9 ? 192 : 96));
  else order_coarse_levels(h);
  // algorithmic work counts
  for (auto& C : h.classes) {
    h.op1_bytes += 16.0 * (C.m + C.nr) * C.m;
    h.se_bytes += 16.0 * C.m * C.m;
    h.phi_bytes += 16.0 * C.m * C.nr;
  }
  for (int e = 0; e < E; ++e) {
    const ElemClass& C = h.classes[h.cls[e]];
    h.flops_F += 8.0 * (C.m + C.nr) * C.m;
    h.flops_P += 4.0 * C.m * C.m;
    h.flops_coarse += 8.0 * C.m * C.nr;
    // the separable solve: four one-index contractions, 4 n^3 flops each with a
    // real eigenbasis acting on complex coefficients, 8 n^3 with a complex one
    bool real_e = true;
    for (auto& v : C.Ex.a) real_e = real_e && v.imag() == 0.0;
    for (auto& v : C.Ey.a) real_e = real_e && v.imag() == 0.0;
    const double n3 = double(C.n) * C.n * C.n;
    h.flops_fdm += (real_e ? 16.0 : 32.0) * n3;
    // its coarse pass: two contractions, the lines i < 2 and j < 2, K_e x_R
    h.flops_fdm_coarse += (real_e ? 8.0 : 16.0) * n3 + 64.0 * C.n * C.n + 8.0 * C.nr * (C.n + C.nr);
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
