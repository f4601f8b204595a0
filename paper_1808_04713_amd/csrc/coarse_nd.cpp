// Nested-dissection multifrontal factor of the coarse matrix K (host side).
//
// The coarse matrix K is factored once per mesh; the paper names that factor
// the method's main cost at high frequency (the dielectric-cylinder example of
// Sec. 3.3.1 and the conclusions).  K couples only coarse unknowns that share
// an element, so with the unknowns in nested-
// dissection order (setup.cpp) block elimination creates fill only inside each
// tree node's front: node t owns the unknowns I (a separator, or a leaf set)
// and, after its subtree is eliminated, couples to the ancestor unknowns B.
// The front F = [F_II F_IB; F_BI F_BB] holds the original entries of the rows
// the node owns plus the children's Schur complements (extend-add); then
//   Dinv = F_II^-1,  L = F_BI Dinv,  S = F_BB - L F_IB  (passed to the parent).
// That is K = L D L^T with D = blockdiag(F_II), so K x = g is solved by
//   forward  (leaves first):  Y_I = front_I,  U = front_B - L Y_I
//   backward (root first):    X_I = Dinv Y_I - L^T X_B.
// Pivoting is partial inside each F_II (Gauss-Jordan); the blocks are taken in
// tree order, as the strip factor takes its strips in order.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <thread>

#include "internal.hpp"

namespace hdp {

namespace {

struct Z {
  double re, im;
};

// C (m x n) += alpha A (m x k) B (k x n), row-major, alpha real.  Four rows of C
// share each row of B.
void zgemm_acc(int m, int n, int k, double alpha, const Z* A, int64_t lda, const Z* B, int64_t ldb, Z* C,
               int64_t ldc) {
  int i = 0;
  for (; i + 4 <= m; i += 4) {
    Z* c0 = C + i * ldc;
    Z* c1 = c0 + ldc;
    Z* c2 = c1 + ldc;
    Z* c3 = c2 + ldc;
    for (int q = 0; q < k; ++q) {
      const Z a0 = A[i * lda + q], a1 = A[(i + 1) * lda + q], a2 = A[(i + 2) * lda + q], a3 = A[(i + 3) * lda + q];
      const double r0 = alpha * a0.re, j0 = alpha * a0.im, r1 = alpha * a1.re, j1 = alpha * a1.im;
      const double r2 = alpha * a2.re, j2 = alpha * a2.im, r3 = alpha * a3.re, j3 = alpha * a3.im;
      const Z* b = B + q * ldb;
      for (int j = 0; j < n; ++j) {
        const double br = b[j].re, bi = b[j].im;
        c0[j].re += r0 * br - j0 * bi; c0[j].im += r0 * bi + j0 * br;
        c1[j].re += r1 * br - j1 * bi; c1[j].im += r1 * bi + j1 * br;
        c2[j].re += r2 * br - j2 * bi; c2[j].im += r2 * bi + j2 * br;
        c3[j].re += r3 * br - j3 * bi; c3[j].im += r3 * bi + j3 * br;
      }
    }
  }
  for (; i < m; ++i) {
    Z* c = C + i * ldc;
    for (int q = 0; q < k; ++q) {
      const Z a = A[i * lda + q];
      const double ar = alpha * a.re, ai = alpha * a.im;
      const Z* b = B + q * ldb;
      for (int j = 0; j < n; ++j) {
        c[j].re += ar * b[j].re - ai * b[j].im;
        c[j].im += ar * b[j].im + ai * b[j].re;
      }
    }
  }
}

// In-place inverse of the n x n row-major A by Gauss-Jordan elimination with
// partial (row) pivoting; false when a pivot column is exactly zero.
bool zinverse(int n, Z* A) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = -1;
    for (int i = k; i < n; ++i) {
      const Z v = A[int64_t(i) * n + k];
      const double m = v.re * v.re + v.im * v.im;
      if (m > best) { best = m; p = i; }
    }
    if (!(best > 0)) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[int64_t(k) * n + j], A[int64_t(p) * n + j]);
    Z* rk = A + int64_t(k) * n;
    const Z d = rk[k];
    const double den = d.re * d.re + d.im * d.im;
    const Z inv{d.re / den, -d.im / den};
    rk[k] = Z{1, 0};
    for (int j = 0; j < n; ++j) {
      const Z v = rk[j];
      rk[j] = Z{v.re * inv.re - v.im * inv.im, v.re * inv.im + v.im * inv.re};
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      Z* ri = A + int64_t(i) * n;
      const Z f = ri[k];
      if (f.re == 0 && f.im == 0) continue;
      ri[k] = Z{0, 0};
      for (int j = 0; j < n; ++j) {
        ri[j].re -= f.re * rk[j].re - f.im * rk[j].im;
        ri[j].im -= f.re * rk[j].im + f.im * rk[j].re;
      }
    }
  }
  for (int k = n - 1; k >= 0; --k)
    if (piv[k] != k)
      for (int i = 0; i < n; ++i) std::swap(A[int64_t(i) * n + k], A[int64_t(i) * n + piv[k]]);
  return true;
}

}  // namespace

void nd_factor(const Handle& h, const std::vector<int64_t>& kidx, const std::vector<double2>& kval, NDHost& f) {
  const int nn = int(h.nd_off.size()) - 1;
  const int64_t nK = h.nK;
  int maxd = 0;
  for (int t = 0; t < nn; ++t) maxd = std::max(maxd, h.nd_depth[t]);
  std::vector<int> node_of(nK);
  for (int t = 0; t < nn; ++t)
    for (int i = h.nd_off[t]; i < h.nd_off[t + 1]; ++i) node_of[i] = t;
  // original entries, each in the front of the node that owns its earlier index
  std::vector<std::vector<int64_t>> bucket(nn);
  for (size_t q = 0; q < kidx.size(); ++q) {
    const int64_t i = kidx[q] % nK, j = kidx[q] / nK;
    bucket[node_of[std::min(i, j)]].push_back(int64_t(q));
  }
  auto nI_of = [&](int t) { return h.nd_off[t + 1] - h.nd_off[t]; };
  auto nB_of = [&](int t) { return int(h.nd_boff[t + 1] - h.nd_boff[t]); };
  // factor layout and update-vector rows
  f.uoff.assign(nn, 0); f.mD.assign(nn, 0); f.mL.assign(nn, 0); f.mLt.assign(nn, 0);
  int64_t tot = 0, urows = 0;
  f.flops_per_col = 0;
  for (int t = 0; t < nn; ++t) {
    const int64_t nI = nI_of(t), nB = nB_of(t);
    f.mD[t] = tot; tot += nI * nI;
    f.mL[t] = tot; tot += nB * nI;
    f.mLt[t] = tot; tot += nI * nB;
    f.uoff[t] = urows; urows += nB;
    f.flops_per_col += 8.0 * double(nI * nI + 2 * nB * nI);
  }
  f.urows = urows;
  f.fac.assign(size_t(tot), make_double2(0, 0));
  Z* fac = reinterpret_cast<Z*>(f.fac.data());
  std::vector<std::vector<Z>> schur(nn);   // S of a node until its parent has used it
  std::vector<std::vector<int>> by_depth(maxd + 1);
  for (int t = 0; t < nn; ++t) by_depth[h.nd_depth[t]].push_back(t);
  std::mutex err_mu;
  std::string err;
  auto factor_node = [&](int t) {
    const int off = h.nd_off[t], nI = nI_of(t), nB = nB_of(t), nf = nI + nB;
    const int* B = h.nd_bnd.data() + h.nd_boff[t];
    auto pos = [&](int64_t g) -> int {
      if (g >= off && g < off + nI) return int(g - off);
      const int* it = std::lower_bound(B, B + nB, int(g));
      if (it == B + nB || *it != g) return -1;
      return nI + int(it - B);
    };
    std::vector<Z> F(size_t(nf) * nf, Z{0, 0});
    for (int64_t q : bucket[t]) {
      const int a = pos(kidx[q] % nK), b = pos(kidx[q] / nK);
      if (a < 0 || b < 0) {
        std::lock_guard<std::mutex> g(err_mu);
        err = "coarse entry outside its nested-dissection front";
        return;
      }
      F[size_t(a) * nf + b].re += kval[q].x;
      F[size_t(a) * nf + b].im += kval[q].y;
    }
    for (int k = 0; k < 2; ++k) {
      const int c = h.nd_child[2 * size_t(t) + k];
      if (c < 0) continue;
      const int nc = nB_of(c);
      const int* Bc = h.nd_bnd.data() + h.nd_boff[c];
      std::vector<int> pc(nc);
      for (int a = 0; a < nc; ++a) {
        pc[a] = pos(Bc[a]);
        if (pc[a] < 0) {
          std::lock_guard<std::mutex> g(err_mu);
          err = "child boundary outside its parent's front";
          return;
        }
      }
      const std::vector<Z>& S = schur[c];
      for (int a = 0; a < nc; ++a)
        for (int b = 0; b < nc; ++b) {
          Z& x = F[size_t(pc[a]) * nf + pc[b]];
          x.re += S[size_t(a) * nc + b].re;
          x.im += S[size_t(a) * nc + b].im;
        }
      std::vector<Z>().swap(schur[c]);
    }
    Z* D = fac + f.mD[t];
    for (int i = 0; i < nI; ++i)
      for (int j = 0; j < nI; ++j) D[size_t(i) * nI + j] = F[size_t(i) * nf + j];
    if (!zinverse(nI, D)) {
      std::lock_guard<std::mutex> g(err_mu);
      err = "singular diagonal block in the nested-dissection coarse factor";
      return;
    }
    if (nB == 0) return;
    Z* L = fac + f.mL[t];
    zgemm_acc(nB, nI, nI, 1.0, F.data() + size_t(nI) * nf, nf, D, nI, L, nI);
    Z* Lt = fac + f.mLt[t];
    for (int b = 0; b < nB; ++b)
      for (int i = 0; i < nI; ++i) Lt[size_t(i) * nB + b] = L[size_t(b) * nI + i];
    std::vector<Z> S(size_t(nB) * nB);
    for (int a = 0; a < nB; ++a)
      for (int b = 0; b < nB; ++b) S[size_t(a) * nB + b] = F[size_t(nI + a) * nf + nI + b];
    zgemm_acc(nB, nB, nI, -1.0, L, nI, F.data() + nI, nf, S.data(), nB);
    schur[t].swap(S);
  };
  const int nthreads = int(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  for (int dpt = maxd; dpt >= 0; --dpt) {
    const std::vector<int>& lv = by_depth[dpt];
    std::atomic<int> next(0);
    auto worker = [&]() {
      for (int q = next++; q < int(lv.size()); q = next++) factor_node(lv[q]);
    };
    const int nt = std::min<int>(nthreads, int(lv.size()));
    std::vector<std::thread> pool;
    for (int k = 1; k < nt; ++k) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    if (!err.empty()) fail(HDP_E_COARSE, err);
  }
  // where each update row goes in the parent's front
  std::vector<int> parent(nn, -1);
  for (int t = 0; t < nn; ++t)
    for (int k = 0; k < 2; ++k)
      if (h.nd_child[2 * size_t(t) + k] >= 0) parent[h.nd_child[2 * size_t(t) + k]] = t;
  // several columns: slot k of the parent's rows for child k (interior rows
  // first, then update rows from nK on)
  f.push.assign(size_t(std::max<int64_t>(1, urows)), 0);
  f.push2.assign(size_t(std::max<int64_t>(1, urows)), 0);
  const int64_t srows = nK + urows;
  if (2 * srows >= (int64_t(1) << 31)) fail(HDP_E_COARSE, "nested-dissection slot index overflows");
  for (int t = 0; t < nn; ++t) {
    const int p = parent[t];
    if (nB_of(t) > 0 && p < 0) fail(HDP_E_COARSE, "nested-dissection root with a boundary");
    const int k = p >= 0 && h.nd_child[2 * size_t(p)] == t ? 0 : 1;
    const int* Bt = h.nd_bnd.data() + h.nd_boff[t];
    for (int a = 0; a < nB_of(t); ++a) {
      const int g = Bt[a];
      if (g >= h.nd_off[p] && g < h.nd_off[p + 1]) {
        f.push[f.uoff[t] + a] = -1 - g;
        f.push2[f.uoff[t] + a] = int(k * srows + g);
      } else {
        const int* Bp = h.nd_bnd.data() + h.nd_boff[p];
        const int* it = std::lower_bound(Bp, Bp + nB_of(p), g);
        if (it == Bp + nB_of(p) || *it != g) fail(HDP_E_COARSE, "child boundary outside its parent's front");
        f.push[f.uoff[t] + a] = int(f.uoff[p] + (it - Bp));
        f.push2[f.uoff[t] + a] = int(k * srows + nK + f.uoff[p] + (it - Bp));
      }
    }
  }
  nd_tasks(h, f, 1024);
}

// Row tasks of the device sweeps, depth by depth.  Several columns: tiles of 32
// outputs; a depth with few tiles splits each tile's sum so that about `target`
// workgroups run (the set-up autotuner tries several targets).
void nd_tasks(const Handle& h, NDHost& f, int target) {
  const int nn = int(h.nd_off.size()) - 1;
  int maxd = 0;
  for (int t = 0; t < nn; ++t) maxd = std::max(maxd, h.nd_depth[t]);
  std::vector<std::vector<int>> by_depth(maxd + 1);
  for (int t = 0; t < nn; ++t) by_depth[h.nd_depth[t]].push_back(t);
  auto nI_of = [&](int t) { return h.nd_off[t + 1] - h.nd_off[t]; };
  auto nB_of = [&](int t) { return int(h.nd_boff[t + 1] - h.nd_boff[t]); };
  f.levels.assign(maxd + 1, NDLevel{});
  f.t1f.clear(); f.t1b.clear(); f.tRf.clear(); f.tRb.clear();
  f.part_tasks = 0;
  for (int dpt = 0; dpt <= maxd; ++dpt) {
    NDLevel& L = f.levels[dpt];
    L.f1 = int(f.t1f.size()); L.b1 = int(f.t1b.size());
    for (int t : by_depth[dpt]) {
      for (int b = 0; b < nB_of(t); ++b) f.t1f.push_back(make_int2(t, b));
      for (int i = 0; i < nI_of(t); ++i) f.t1b.push_back(make_int2(t, i));
    }
    L.nf1 = int(f.t1f.size()) - L.f1; L.nb1 = int(f.t1b.size()) - L.b1;
    for (int bwd = 0; bwd < 2; ++bwd) {
      int ntiles = 0, kmax = 0;
      for (int t : by_depth[dpt]) {
        const int nout = bwd ? nI_of(t) : nB_of(t);
        ntiles += (nout + 31) / 32;
        if (nout > 0) kmax = std::max(kmax, bwd ? nI_of(t) + nB_of(t) : nI_of(t));
      }
      int S = 1;
      if (ntiles > 0) S = std::max(1, std::min((target + ntiles - 1) / ntiles, (kmax + 31) / 32));
      std::vector<int4>& T = bwd ? f.tRb : f.tRf;
      const int first = int(T.size());
      // nodes with the longest sums first: a depth whose tiles overflow one round
      // of workgroups leaves its shortest ones for the last round (each output's
      // tasks stay together, so every sum is the same)
      std::vector<int> order = by_depth[dpt];
      std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        const int ka = bwd ? nI_of(a) + nB_of(a) : nI_of(a), kc = bwd ? nI_of(c) + nB_of(c) : nI_of(c);
        return ka > kc;
      });
      for (int t : order) {
        const int nout = bwd ? nI_of(t) : nB_of(t);
        const int K = bwd ? nI_of(t) + nB_of(t) : nI_of(t);
        const int chunk = (K + S - 1) / S;
        for (int j = 0; j < nout; j += 32)
          for (int c = 0; c < S; ++c) {
            const int i0 = std::min(K, c * chunk), i1 = std::min(K, (c + 1) * chunk);
            T.push_back(make_int4(t, j, i0, i1));
          }
      }
      if (S > 1) f.part_tasks = std::max<int64_t>(f.part_tasks, int64_t(ntiles) * S);
      if (bwd) { L.bR = first; L.nbR = ntiles; L.Sb = S; }
      else { L.fR = first; L.nfR = ntiles; L.Sf = S; }
    }
  }
}

}  // namespace hdp
