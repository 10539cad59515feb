// Stiefel manifold, preconditioner, L-BFGS and the optimisation driver (see optim.h).
#include "optim.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>

#include "linalg.h"
#include "vec.h"

namespace mera {

namespace {

VPtr d64(const MatView& m) { return VPtr{m.data, Prec::F64}; }
int64_t numel(const MatView& m) { return (int64_t)m.n * m.p; }
double* tmp(Ctx& ctx, const std::string& name, int64_t n) {
  return static_cast<double*>(ctx.buf(name, (size_t)n * sizeof(double)));
}

}  // namespace

void Flat::init(const std::vector<int>& n_, const std::vector<int>& p_) {
  n = n_;
  p = p_;
  off.assign(n.size(), 0);
  total = 0;
  for (size_t i = 0; i < n.size(); ++i) {
    off[i] = total;
    total += (int64_t)n[i] * p[i];
  }
  buf.alloc((size_t)std::max<int64_t>(total, 1) * sizeof(double));
}

std::vector<MatView> Flat::views() const {
  std::vector<MatView> v;
  for (int i = 0; i < count(); ++i) v.push_back(view(i));
  return v;
}

double inner(Ctx& ctx, const std::vector<MatView>& X, const std::vector<MatView>& Y) {
  const size_t k = X.size();
  std::vector<VPtr> x(k), y(k);
  std::vector<int64_t> n(k);
  std::vector<double> d(k);
  for (size_t i = 0; i < k; ++i) {
    x[i] = d64(X[i]);
    y[i] = d64(Y[i]);
    n[i] = numel(X[i]);
  }
  dots(ctx, x.data(), y.data(), n.data(), (int)k, d.data());
  double s = 0.0;
  for (size_t i = 0; i < k; ++i) s += d[i];
  return s;
}

void stiefel_project_one(Ctx& ctx, const MatView& W, const MatView& D, const MatView& G) {
  const int n = W.n, p = W.p;
  double* S = tmp(ctx, "st.S", (int64_t)p * p);
  mm(ctx, "S[pq] = W[np] * D[nq]", {{'n', n}, {'p', p}, {'q', p}}, {{"S", S}, {"W", W.data}, {"D", D.data}});
  symmetrize(ctx, VPtr{S, Prec::F64}, p);
  if (G.data != D.data) copy(ctx, d64(G), d64(D), (int64_t)n * p);
  mm(ctx, "G[nq] += -1.0 * W[np] * S[pq]", {{'n', n}, {'p', p}, {'q', p}},
     {{"G", G.data}, {"W", W.data}, {"S", S}});
}

void project_many(Ctx& ctx, const std::vector<MatView>& W, const std::vector<MatView>& D,
                  const std::vector<MatView>& G, const std::vector<bool>& grassmann) {
  // items of equal shape run in grouped launches; each item computes what stiefel_project_one (or
  // grassmann_project_one) computes for it alone
  const size_t k = W.size();
  std::vector<bool> done(k, false);
  for (size_t a = 0; a < k; ++a) {
    if (done[a]) continue;
    std::vector<size_t> grp;
    for (size_t b = a; b < k && grp.size() < (size_t)kGettMaxGroup; ++b)
      if (!done[b] && W[b].n == W[a].n && W[b].p == W[a].p) {
        grp.push_back(b);
        done[b] = true;
      }
    const int n = W[a].n, p = W[a].p;
    std::vector<std::vector<void*>> s1, s2;
    std::vector<double*> S(grp.size());
    for (size_t j = 0; j < grp.size(); ++j) {
      S[j] = tmp(ctx, "pj.S" + std::to_string(j), (int64_t)p * p);
      s1.push_back({S[j], W[grp[j]].data, D[grp[j]].data});
    }
    mm_group(ctx, "S[pq] = W[np] * D[nq]", {{'n', n}, {'p', p}, {'q', p}}, {"S", "W", "D"}, s1);
    for (size_t j = 0; j < grp.size(); ++j) {
      const size_t i = grp[j];
      if (!grassmann[i]) symmetrize(ctx, VPtr{S[j], Prec::F64}, p);
      if (G[i].data != D[i].data) copy(ctx, d64(G[i]), d64(D[i]), (int64_t)n * p);
      s2.push_back({G[i].data, W[i].data, S[j]});
    }
    mm_group(ctx, "G[nq] += -1.0 * W[np] * S[pq]", {{'n', n}, {'p', p}, {'q', p}}, {"G", "W", "S"}, s2);
  }
}

void stiefel_retract_many(Ctx& ctx, const std::vector<MatView>& W, const std::vector<MatView>& X, double alpha,
                          const std::vector<MatView>& Wout, const std::vector<const MatView*>& Xout) {
  // Every factor runs the same sequence of operations as it would alone; the factors step through the
  // Newton-Schulz iteration together, so that the convergence norms of all of them come back in one
  // synchronisation per step. Scratch is per factor.
  const size_t k = W.size();
  struct Fac {
    int n, p;
    int64_t pp;
    double *Y, *M, *Yk, *Zk, *Tk, *Y2, *Z2;
    double c = 0.0;
    int tail = 0;
    bool conv = false;
  };
  std::vector<Fac> fs(k);
  for (size_t i = 0; i < k; ++i) {
    Fac& f = fs[i];
    f.n = W[i].n;
    f.p = W[i].p;
    f.pp = (int64_t)f.p * f.p;
    const std::string t = std::to_string(i);
    f.Y = tmp(ctx, "rt.Y" + t, (int64_t)f.n * f.p);
    f.M = tmp(ctx, "rt.M" + t, f.pp);
    f.Yk = tmp(ctx, "rt.Yk" + t, f.pp);
    f.Zk = tmp(ctx, "rt.Zk" + t, f.pp);
    f.Tk = tmp(ctx, "rt.T" + t, f.pp);
    f.Y2 = tmp(ctx, "rt.Y2" + t, f.pp);
    f.Z2 = tmp(ctx, "rt.Z2" + t, f.pp);
    copy(ctx, VPtr{f.Y, Prec::F64}, d64(W[i]), (int64_t)f.n * f.p);
    axpby(ctx, alpha, d64(X[i]), 1.0, VPtr{f.Y, Prec::F64}, (int64_t)f.n * f.p);
    // M = Y^T Y
    mm(ctx, "M[pq] = Y[np] * Y2[nq]", {{'n', f.n}, {'p', f.p}, {'q', f.p}}, {{"M", f.M}, {"Y", f.Y}, {"Y2", f.Y}});
    symmetrize(ctx, VPtr{f.M, Prec::F64}, f.p);
  }
  // coupled Newton-Schulz iteration (Higham, "Functions of Matrices", the coupled square-root iteration):
  // Y_0 = M/c, Z_0 = I, T = (3I - Z Y)/2, Y <- Y T, Z <- T Z; Z -> (M/c)^{-1/2}
  std::vector<VPtr> xa(k);
  std::vector<int64_t> na(k);
  std::vector<double> d(k);
  for (size_t i = 0; i < k; ++i) {
    xa[i] = VPtr{fs[i].M, Prec::F64};
    na[i] = fs[i].pp;
  }
  dots(ctx, xa.data(), xa.data(), na.data(), (int)k, d.data());
  for (size_t i = 0; i < k; ++i) {
    Fac& f = fs[i];
    f.c = std::sqrt(d[i]);
    MERA_CHECK(std::isfinite(f.c) && f.c > 0.0, MERA_ENONFINITE, "retraction: non-finite Y^T Y");
    copy(ctx, VPtr{f.Yk, Prec::F64}, VPtr{f.M, Prec::F64}, f.pp);
    scal(ctx, 1.0 / f.c, VPtr{f.Yk, Prec::F64}, f.pp);
    fill(ctx, VPtr{f.Zk, Prec::F64}, f.pp, 0.0);
    add_diag(ctx, VPtr{f.Zk, Prec::F64}, f.p, 1.0);
  }
  std::vector<size_t> active(k);
  for (size_t i = 0; i < k; ++i) active[i] = i;
  for (int it = 0; it < 100 && !active.empty(); ++it) {
    // one step for every active factor; factors of equal size share grouped launches
    std::vector<bool> stepped(active.size(), false);
    for (size_t a = 0; a < active.size(); ++a) {
      if (stepped[a]) continue;
      std::vector<Fac*> g;
      for (size_t b = a; b < active.size() && g.size() < (size_t)kGettMaxGroup; ++b)
        if (!stepped[b] && fs[active[b]].p == fs[active[a]].p) {
          g.push_back(&fs[active[b]]);
          stepped[b] = true;
        }
      const int p = g[0]->p;
      const std::initializer_list<std::pair<char, int64_t>> dpp = {{'p', p}, {'q', p}, {'r', p}};
      std::vector<std::vector<void*>> b1, b2, b3;
      for (Fac* f : g) b1.push_back({f->Tk, f->Zk, f->Yk});
      mm_group(ctx, "T[pq] = -0.5 * Z[pr] * Yk[rq]", dpp, {"T", "Z", "Yk"}, b1);
      for (Fac* f : g) {
        add_diag(ctx, VPtr{f->Tk, Prec::F64}, p, 1.5);
        b2.push_back({f->Y2, f->Yk, f->Tk});
        b3.push_back({f->Z2, f->Tk, f->Zk});
      }
      mm_group(ctx, "Y2[pq] = Yk[pr] * T[rq]", dpp, {"Y2", "Yk", "T"}, b2);
      mm_group(ctx, "Z2[pq] = T[pr] * Z[rq]", dpp, {"Z2", "T", "Z"}, b3);
      for (Fac* f : g) {
        std::swap(f->Yk, f->Y2);
        std::swap(f->Zk, f->Z2);
        add_diag(ctx, VPtr{f->Tk, Prec::F64}, p, -1.0);
      }
    }
    const size_t na_ = active.size();
    for (size_t j = 0; j < na_; ++j) {
      xa[j] = VPtr{fs[active[j]].Tk, Prec::F64};
      na[j] = fs[active[j]].pp;
    }
    dots(ctx, xa.data(), xa.data(), na.data(), (int)na_, d.data());
    std::vector<size_t> still;
    for (size_t j = 0; j < na_; ++j) {
      Fac& f = fs[active[j]];
      const double err = std::sqrt(d[j]);
      MERA_CHECK(std::isfinite(err), MERA_ENONFINITE, "retraction: Newton-Schulz diverged");
      // quadratic convergence: one more step after the first below 1e-13 reaches rounding level
      if (err < 1e-13 && ++f.tail >= 2) f.conv = true;
      else still.push_back(active[j]);
    }
    active.swap(still);
  }
  for (const Fac& f : fs) MERA_CHECK(f.conv, MERA_ENOCONV, "retraction: Newton-Schulz did not converge");
  for (size_t i = 0; i < k; ++i) {
    Fac& f = fs[i];
    const int n = f.n, p = f.p;
    const int64_t pp = f.pp;
    const std::initializer_list<std::pair<char, int64_t>> dpp = {{'p', p}, {'q', p}, {'r', p}};
    // Z = M^{-1/2}
    scal(ctx, 1.0 / std::sqrt(f.c), VPtr{f.Zk, Prec::F64}, pp);
    double* Wt = tmp(ctx, "rt.W", (int64_t)n * p);
    mm(ctx, "Wt[nq] = Y[np] * Z[pq]", {{'n', n}, {'p', p}, {'q', p}}, {{"Wt", Wt}, {"Y", f.Y}, {"Z", f.Zk}});
    // one Newton-Schulz polar refinement: W <- W (3I - W^T W)/2
    mm(ctx, "E[pq] = Wt[np] * Wt2[nq]", {{'n', n}, {'p', p}, {'q', p}}, {{"E", f.Tk}, {"Wt", Wt}, {"Wt2", Wt}});
    scal(ctx, -0.5, VPtr{f.Tk, Prec::F64}, pp);
    add_diag(ctx, VPtr{f.Tk, Prec::F64}, p, 1.5);
    mm(ctx, "Wo[nq] = Wt[np] * E[pq]", {{'n', n}, {'p', p}, {'q', p}},
       {{"Wo", Wout[i].data}, {"Wt", Wt}, {"E", f.Tk}});
    if (Xout[i]) {
      // M = I + alpha^2 K with K = X^T X (X tangent), and M commutes with K, so
      // dR/dalpha = X Z + (W + alpha X) dZ/dalpha = X Z - alpha Y K Z^3.
      double* K = tmp(ctx, "rt.K", pp);
      mm(ctx, "K[pq] = X[np] * X2[nq]", {{'n', n}, {'p', p}, {'q', p}}, {{"K", K}, {"X", X[i].data}, {"X2", X[i].data}});
      mm(ctx, "Y2[pq] = Z[pr] * Z2[rq]", dpp, {{"Y2", f.Y2}, {"Z", f.Zk}, {"Z2", f.Zk}});    // Z^2
      mm(ctx, "T[pq] = Y2[pr] * Z[rq]", dpp, {{"T", f.Tk}, {"Y2", f.Y2}, {"Z", f.Zk}});      // Z^3
      mm(ctx, "Y2[pq] = K[pr] * T[rq]", dpp, {{"Y2", f.Y2}, {"K", K}, {"T", f.Tk}});         // K Z^3
      scal(ctx, -alpha, VPtr{f.Y2, Prec::F64}, pp);
      mm(ctx, "Xo[nq] = X[np] * Z[pq]", {{'n', n}, {'p', p}, {'q', p}},
         {{"Xo", Xout[i]->data}, {"X", X[i].data}, {"Z", f.Zk}});
      mm(ctx, "Xo[nq] += Y[np] * KZ[pq]", {{'n', n}, {'p', p}, {'q', p}},
         {{"Xo", Xout[i]->data}, {"Y", f.Y}, {"KZ", f.Y2}});
    }
  }
}

void stiefel_retract_one(Ctx& ctx, const MatView& W, const MatView& X, double alpha, const MatView& Wout,
                         const MatView* Xout) {
  stiefel_retract_many(ctx, {W}, {X}, alpha, {Wout}, {Xout});
}

void grassmann_project_one(Ctx& ctx, const MatView& W, const MatView& D, const MatView& G) {
  const int n = W.n, p = W.p;
  double* S = tmp(ctx, "gp.S", (int64_t)p * p);
  mm(ctx, "S[pq] = W[np] * D[nq]", {{'n', n}, {'p', p}, {'q', p}}, {{"S", S}, {"W", W.data}, {"D", D.data}});
  if (G.data != D.data) copy(ctx, d64(G), d64(D), (int64_t)n * p);
  mm(ctx, "G[nq] += -1.0 * W[np] * S[pq]", {{'n', n}, {'p', p}, {'q', p}},
     {{"G", G.data}, {"W", W.data}, {"S", S}});
}

// ---- exponential retraction and transport (Sec. 2.3) -------------------------------------------------------

void exp_frame_one(Ctx& ctx, const MatView& W, const MatView& X, ExpFrame& fr) {
  const int n = W.n, p = W.p;
  const int r = std::min(p, n - p);
  fr.n = n;
  fr.p = p;
  fr.m = r > 0 ? 2 * p : p;
  fr.has_alpha = false;
  const int m = fr.m;
  fr.M.ensure((size_t)m * m * 8);
  fr.E.ensure((size_t)m * m * 8);
  double* M = fr.M.as<double>();
  const std::initializer_list<std::pair<char, int64_t>> dnp = {{'n', n}, {'p', p}, {'q', p}};
  double* A = tmp(ctx, "ex.A", (int64_t)p * p);
  mm(ctx, "A[pq] = W[np] * X[nq]", dnp, {{"A", A}, {"W", W.data}, {"X", X.data}});
  fill(ctx, VPtr{M, Prec::F64}, (int64_t)m * m, 0.0);
  copy_block(ctx, M, m, A, p, p, p, 1.0);
  if (r == 0) return;
  // Z = (1 - W W^T) X; an orthonormal basis of range(Z) from the eigendecomposition of Z^T Z (any basis gives the
  // same exp(alpha Q_X)): Q = Z V_r diag(lam_r^{-1/2}) over the r largest eigenvalues above rounding
  fr.Q.ensure((size_t)n * p * 8);
  double* Q = fr.Q.as<double>();
  double* Z = tmp(ctx, "ex.Z", (int64_t)n * p);
  copy(ctx, VPtr{Z, Prec::F64}, d64(X), (int64_t)n * p);
  mm(ctx, "Z[nq] += -1.0 * W[np] * A[pq]", dnp, {{"Z", Z}, {"W", W.data}, {"A", A}});
  double* K = tmp(ctx, "ex.K", (int64_t)p * p);
  mm(ctx, "K[pq] = Z[np] * Z2[nq]", dnp, {{"K", K}, {"Z", Z}, {"Z2", Z}});
  symmetrize(ctx, VPtr{K, Prec::F64}, p);
  double* lam = tmp(ctx, "ex.lam", p);
  double* V = tmp(ctx, "ex.V", (int64_t)p * p);
  jacobi_eigh(ctx, K, lam, V, p);
  std::vector<double> hl(p), sc(p, 0.0);
  MERA_HIP(hipMemcpyAsync(hl.data(), lam, (size_t)p * 8, hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();
  std::vector<int> order(p);
  for (int i = 0; i < p; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return hl[a] > hl[b]; });
  const double lmax = hl[order[0]];
  for (int k = 0; k < r; ++k) {
    const int i = order[k];
    if (lmax > 0.0 && hl[i] > 1e-24 * lmax) sc[i] = 1.0 / std::sqrt(hl[i]);
  }
  double* sdev = tmp(ctx, "ex.s", p);
  MERA_HIP(hipMemcpyAsync(sdev, sc.data(), (size_t)p * 8, hipMemcpyHostToDevice, ctx.stream));
  mm(ctx, "Q[nq] = Z[np] * V[pq]", dnp, {{"Q", Q}, {"Z", Z}, {"V", V}});
  scale_cols(ctx, Q, sdev, n, p);
  ctx.sync();  // sc is host memory read by the copy above
  double* B = tmp(ctx, "ex.B", (int64_t)p * p);
  double* BT = tmp(ctx, "ex.BT", (int64_t)p * p);
  mm(ctx, "B[pq] = Q[np] * Z[nq]", dnp, {{"B", B}, {"Q", Q}, {"Z", Z}});
  mm(ctx, "BT[pq] = Z[np] * Q[nq]", dnp, {{"BT", BT}, {"Z", Z}, {"Q", Q}});
  copy_block(ctx, M + (int64_t)p * m, m, B, p, p, p, 1.0);   // lower left:  B
  copy_block(ctx, M + p, m, BT, p, p, p, -1.0);              // upper right: -B^T
}

void exp_set_alpha(Ctx& ctx, ExpFrame& fr, double alpha) {
  const int m = fr.m;
  const int64_t mm2 = (int64_t)m * m;
  const double* M = fr.M.as<double>();
  const double nrm = std::fabs(alpha) * std::sqrt(dot(ctx, VPtr{(void*)M, Prec::F64}, VPtr{(void*)M, Prec::F64}, mm2));
  MERA_CHECK(std::isfinite(nrm), MERA_ENONFINITE, "exponential retraction: non-finite generator");
  // scaling and squaring: ||alpha M / 2^s||_F <= 1/2, Taylor polynomial of degree 14 (remainder below 3e-17)
  int s = 0;
  while (nrm > 0.5 * std::ldexp(1.0, s) && s < 60) ++s;
  const double c = alpha * std::ldexp(1.0, -s);
  double* Bm = tmp(ctx, "ex.Bm", mm2);
  double* P = tmp(ctx, "ex.P", mm2);
  double* T = tmp(ctx, "ex.T", mm2);
  copy(ctx, VPtr{Bm, Prec::F64}, VPtr{(void*)M, Prec::F64}, mm2);
  scal(ctx, c, VPtr{Bm, Prec::F64}, mm2);
  const std::initializer_list<std::pair<char, int64_t>> dmm = {{'i', m}, {'j', m}, {'l', m}};
  constexpr int kDeg = 14;
  copy(ctx, VPtr{P, Prec::F64}, VPtr{Bm, Prec::F64}, mm2);
  scal(ctx, 1.0 / kDeg, VPtr{P, Prec::F64}, mm2);
  add_diag(ctx, VPtr{P, Prec::F64}, m, 1.0);
  for (int k = kDeg - 1; k >= 1; --k) {  // Horner: P <- 1 + B P / k
    mm(ctx, "T[ij] = B[il] * P[lj]", dmm, {{"T", T}, {"B", Bm}, {"P", P}});
    scal(ctx, 1.0 / k, VPtr{T, Prec::F64}, mm2);
    add_diag(ctx, VPtr{T, Prec::F64}, m, 1.0);
    std::swap(P, T);
  }
  for (int i = 0; i < s; ++i) {
    mm(ctx, "T[ij] = P[il] * P2[lj]", dmm, {{"T", T}, {"P", P}, {"P2", P}});
    std::swap(P, T);
  }
  copy(ctx, VPtr{fr.E.ptr, Prec::F64}, VPtr{P, Prec::F64}, mm2);
  fr.alpha = alpha;
  fr.has_alpha = true;
}

void exp_apply_one(Ctx& ctx, const MatView& W, const ExpFrame& fr, const MatView& Y, const MatView& out) {
  const int n = fr.n, p = fr.p, m = fr.m;
  MERA_CHECK(fr.has_alpha && W.n == n && W.p == p && Y.n == n && Y.p == p, MERA_EINVAL, "exponential transport");
  const std::initializer_list<std::pair<char, int64_t>> dnp = {{'n', n}, {'p', p}, {'q', p}};
  double* C = tmp(ctx, "ea.C", (int64_t)m * p);
  double* D = tmp(ctx, "ea.D", (int64_t)m * p);
  double* Em = tmp(ctx, "ea.Em", (int64_t)m * m);
  const bool low = m == 2 * p;
  // C = U^T Y = [W^T Y; Q^T Y]
  mm(ctx, "C[pq] = W[np] * Y[nq]", dnp, {{"C", C}, {"W", W.data}, {"Y", Y.data}});
  if (low) mm(ctx, "C[pq] = Q[np] * Y[nq]", dnp, {{"C", C + (int64_t)p * p}, {"Q", fr.Q.ptr}, {"Y", Y.data}});
  // D = (E - 1) C
  copy(ctx, VPtr{Em, Prec::F64}, VPtr{fr.E.ptr, Prec::F64}, (int64_t)m * m);
  add_diag(ctx, VPtr{Em, Prec::F64}, m, -1.0);
  mm(ctx, "D[iq] = Em[ij] * C[jq]", {{'i', m}, {'j', m}, {'q', p}}, {{"D", D}, {"Em", Em}, {"C", C}});
  // out = Y + U D
  if (out.data != Y.data) copy(ctx, d64(out), d64(Y), (int64_t)n * p);
  mm(ctx, "O[nq] += W[np] * D[pq]", dnp, {{"O", out.data}, {"W", W.data}, {"D", D}});
  if (low) mm(ctx, "O[nq] += Q[np] * D[pq]", dnp, {{"O", out.data}, {"Q", fr.Q.ptr}, {"D", D + (int64_t)p * p}});
}

void exp_retract_one(Ctx& ctx, const MatView& W, const MatView& X, ExpFrame& fr, double alpha, const MatView& Wout,
                     const MatView* Xout) {
  const int n = W.n, p = W.p;
  if (!fr.has_alpha || fr.alpha != alpha) exp_set_alpha(ctx, fr, alpha);
  if (Xout) exp_apply_one(ctx, W, fr, X, *Xout);
  double* Wt = tmp(ctx, "er.W", (int64_t)n * p);
  exp_apply_one(ctx, W, fr, W, MatView{n, p, Wt});
  // one Newton-Schulz polar refinement: W <- W (3 - W^T W)/2
  double* S = tmp(ctx, "er.S", (int64_t)p * p);
  mm(ctx, "S[pq] = Wt[np] * Wt2[nq]", {{'n', n}, {'p', p}, {'q', p}}, {{"S", S}, {"Wt", Wt}, {"Wt2", Wt}});
  scal(ctx, -0.5, VPtr{S, Prec::F64}, (int64_t)p * p);
  add_diag(ctx, VPtr{S, Prec::F64}, p, 1.5);
  mm(ctx, "Wo[nq] = Wt[np] * S[pq]", {{'n', n}, {'p', p}, {'q', p}}, {{"Wo", Wout.data}, {"Wt", Wt}, {"S", S}});
}

// ---- Evenbly-Vidal update (App. A) ------------------------------------------------------------------------

void ev_update_one(Ctx& ctx, const MatView& W, const MatView& D, const MatView& rho, double gamma,
                   const MatView& Wout) {
  const int n = W.n, p = W.p;
  const int64_t np_ = (int64_t)n * p, pp = (int64_t)p * p;
  const std::initializer_list<std::pair<char, int64_t>> dnp = {{'n', n}, {'p', p}, {'q', p}};
  const std::initializer_list<std::pair<char, int64_t>> dpp = {{'p', p}, {'q', p}, {'r', p}};
  double* Y = tmp(ctx, "ev.Y", np_);
  mm(ctx, "Y[nq] = W[np] * R[pq]", dnp, {{"Y", Y}, {"W", W.data}, {"R", rho.data}});
  axpby(ctx, -1.0, d64(D), gamma, VPtr{Y, Prec::F64}, np_);   // Y = gamma W rho - D
  double* K = tmp(ctx, "ev.K", pp);
  double* lam = tmp(ctx, "ev.lam", p);
  double* V = tmp(ctx, "ev.V", pp);
  std::vector<double> hl(p);
  double lmax = 0.0;
  // Y^T Y = V diag(lam) V^T; returns whether Y has full column rank
  auto gram = [&]() {
    mm(ctx, "K[pq] = Y[np] * Y2[nq]", dnp, {{"K", K}, {"Y", Y}, {"Y2", Y}});
    symmetrize(ctx, VPtr{K, Prec::F64}, p);
    jacobi_eigh(ctx, K, lam, V, p);
    MERA_HIP(hipMemcpyAsync(hl.data(), lam, (size_t)p * 8, hipMemcpyDeviceToHost, ctx.stream));
    ctx.sync();
    lmax = 0.0;
    for (double x : hl) {
      MERA_CHECK(std::isfinite(x), MERA_ENONFINITE, "Evenbly-Vidal update: non-finite environment");
      lmax = std::max(lmax, x);
    }
    MERA_CHECK(lmax > 0.0, MERA_ENONFINITE, "Evenbly-Vidal update: gamma W rho - D vanishes");
    for (double x : hl)
      if (!(x > 1e-24 * lmax)) return false;
    return true;
  };
  int refine = 1;  // Newton-Schulz polar refinements after the eigenvalue step
  if (!gram()) {
    // A rank-deficient Y has many polar factors. Take the limit of polar(Y + delta W) for small delta: on Y's
    // range it is Y's own polar factor, on the null space it keeps W's columns. Y + delta W is ill-conditioned
    // (about 1e7), so the eigenvalue step is followed by more refinements (each squares the isometry error).
    axpby(ctx, 1e-7 * std::sqrt(lmax), VPtr{W.data, Prec::F64}, 1.0, VPtr{Y, Prec::F64}, np_);
    MERA_CHECK(gram(), MERA_ENONFINITE, "Evenbly-Vidal update: gamma W rho - D is rank deficient");
    refine = 4;
  }
  for (double& x : hl) x = 1.0 / std::sqrt(x);
  double* sdev = tmp(ctx, "ev.s", p);
  MERA_HIP(hipMemcpyAsync(sdev, hl.data(), (size_t)p * 8, hipMemcpyHostToDevice, ctx.stream));
  double* T = tmp(ctx, "ev.T", pp);
  double* Z = tmp(ctx, "ev.Z", pp);
  copy(ctx, VPtr{T, Prec::F64}, VPtr{V, Prec::F64}, pp);
  scale_cols(ctx, T, sdev, p, p);
  ctx.sync();  // hl is host memory read by the copy above
  mm(ctx, "Z[pq] = T[pr] * V[qr]", dpp, {{"Z", Z}, {"T", T}, {"V", V}});   // (Y^T Y)^{-1/2}
  double* Wt = tmp(ctx, "ev.W", np_);
  mm(ctx, "Wt[nq] = Y[np] * Z[pq]", dnp, {{"Wt", Wt}, {"Y", Y}, {"Z", Z}});
  // Newton-Schulz polar refinements W <- W (3 - W^T W)/2, the last one into Wout
  for (int r = 0; r < refine; ++r) {
    mm(ctx, "S[pq] = Wt[np] * Wt2[nq]", dnp, {{"S", T}, {"Wt", Wt}, {"Wt2", Wt}});
    scal(ctx, -0.5, VPtr{T, Prec::F64}, pp);
    add_diag(ctx, VPtr{T, Prec::F64}, p, 1.5);
    double* dst = (r + 1 == refine) ? Wout.data : Y;  // Y is no longer needed
    mm(ctx, "Wo[nq] = Wt[np] * S[pq]", dnp, {{"Wo", dst}, {"Wt", Wt}, {"S", T}});
    if (r + 1 < refine) copy(ctx, VPtr{Wt, Prec::F64}, VPtr{Y, Prec::F64}, np_);
  }
}

// The density matrices of consecutive iterates differ little, so the previous eigenbasis Q nearly diagonalises the
// new rho: the decomposition starts from Q^T rho Q and needs a few Jacobi sweeps instead of a full run. One in
// kMetricColdEvery decompositions starts from scratch, which keeps the accumulated rounding in Q's orthogonality
// bounded.
constexpr int kMetricColdEvery = 32;

void Metric::compute(Ctx& ctx, const std::vector<MatView>& rho) {
  const size_t k = rho.size();
  const std::vector<int> prev_p = p;
  V.resize(k);
  lam.resize(k);
  f.resize(k);
  g.resize(k);
  warm.resize(k, 0);
  p.assign(k, 0);
  // every factor's matrix is prepared first (each in its own scratch), then all are decomposed together: the
  // small ones (p <= 64) in one launch, one workgroup each
  std::vector<JacobiTask> tasks;
  tasks.reserve(k);
  std::vector<std::pair<size_t, double*>> rotate;  // warm-started factors and their symmetrised rho
  for (size_t i = 0; i < k; ++i) {
    const int q = rho[i].p;
    MERA_CHECK(rho[i].n == q, MERA_EINVAL, "metric must be square");
    const bool reuse = i < prev_p.size() && prev_p[i] == q && warm[i] > 0 && warm[i] < kMetricColdEvery &&
                       V[i].bytes >= (size_t)q * q * 8;
    p[i] = q;
    V[i].ensure((size_t)q * q * 8);
    lam[i].ensure((size_t)q * 8);
    f[i].ensure((size_t)q * 8);
    g[i].ensure((size_t)q * 8);
    const std::string tag = std::to_string(i);
    double* a = tmp(ctx, "met.a" + tag, (int64_t)q * q);
    copy(ctx, VPtr{a, Prec::F64}, d64(rho[i]), (int64_t)q * q);
    symmetrize(ctx, VPtr{a, Prec::F64}, q);
    double* Q = V[i].as<double>();
    if (reuse) {
      double* b = tmp(ctx, "met.b" + tag, (int64_t)q * q);
      tasks.push_back(JacobiTask{b, lam[i].as<double>(), Q, q, 1e-15, 30, true});
      rotate.push_back({i, a});
      warm[i]++;
    } else {
      tasks.push_back(JacobiTask{a, lam[i].as<double>(), Q, q});
      warm[i] = 1;
    }
  }
  // B = Q^T A Q for the warm-started factors, those of equal size in grouped launches
  std::vector<bool> done(rotate.size(), false);
  for (size_t a0 = 0; a0 < rotate.size(); ++a0) {
    if (done[a0]) continue;
    const int q = p[rotate[a0].first];
    std::vector<std::vector<void*>> s1, s2;
    std::vector<double*> bs;
    for (size_t b0 = a0; b0 < rotate.size() && s1.size() < (size_t)kGettMaxGroup; ++b0) {
      const size_t i = rotate[b0].first;
      if (done[b0] || p[i] != q) continue;
      done[b0] = true;
      const std::string tag = std::to_string(i);
      double* t = tmp(ctx, "met.t" + tag, (int64_t)q * q);
      double* b = tmp(ctx, "met.b" + tag, (int64_t)q * q);
      double* Q = V[i].as<double>();
      s1.push_back({t, rotate[b0].second, Q});
      s2.push_back({b, Q, t});
      bs.push_back(b);
    }
    const std::initializer_list<std::pair<char, int64_t>> dpp = {{'p', q}, {'q', q}, {'r', q}};
    mm_group(ctx, "T[pq] = A[pr] * Q[rq]", dpp, {"T", "A", "Q"}, s1);
    mm_group(ctx, "B[pq] = Q[rp] * T[rq]", dpp, {"B", "Q", "T"}, s2);
    for (double* b : bs) symmetrize(ctx, VPtr{b, Prec::F64}, q);
  }
  jacobi_eigh_batch(ctx, tasks);
}

void precondition_one(Ctx& ctx, const MatView& W, const MatView& X, Metric& met, int i, double delta,
                      const MatView& Xout) {
  const int n = W.n, p = W.p;
  MERA_CHECK(met.p[i] == p, MERA_EINVAL, "metric size does not match the tensor");
  if (delta < 0) delta = std::sqrt(dot(ctx, d64(X), d64(X), (int64_t)n * p));
  double* V = met.V[i].as<double>();
  double* f = met.f[i].as<double>();
  double* g = met.g[i].as<double>();
  reg_spectrum(ctx, met.lam[i].as<double>(), delta, f, g, p);
  const int64_t pp = (int64_t)p * p;
  double* A = tmp(ctx, "pc.A", pp);
  double* T1 = tmp(ctx, "pc.T1", pp);
  double* Ah = tmp(ctx, "pc.Ah", pp);
  double* Bp = tmp(ctx, "pc.B", (int64_t)n * p);
  double* T3 = tmp(ctx, "pc.T3", (int64_t)n * p);
  const std::initializer_list<std::pair<char, int64_t>> dpp = {{'p', p}, {'q', p}, {'r', p}};
  const std::initializer_list<std::pair<char, int64_t>> dnp = {{'n', n}, {'p', p}, {'q', p}};
  // A = W^T X; X = W A + (X - W A) with (X - W A) = W_perp B
  mm(ctx, "A[pq] = W[np] * X[nq]", dnp, {{"A", A}, {"W", W.data}, {"X", X.data}});
  copy(ctx, VPtr{Bp, Prec::F64}, d64(X), (int64_t)n * p);
  mm(ctx, "B[nq] += -1.0 * W[np] * A[pq]", dnp, {{"B", Bp}, {"W", W.data}, {"A", A}});
  // A~ = V [ (V^T A V)_ij 2 / (f_i + f_j) ] V^T
  mm(ctx, "T1[pq] = V[rp] * A[rq]", dpp, {{"T1", T1}, {"V", V}, {"A", A}});
  mm(ctx, "Ah[pq] = T1[pr] * V[rq]", dpp, {{"Ah", Ah}, {"T1", T1}, {"V", V}});
  scale_sylvester(ctx, Ah, f, p);
  mm(ctx, "T1[pq] = V[pr] * Ah[rq]", dpp, {{"T1", T1}, {"V", V}, {"Ah", Ah}});
  mm(ctx, "A[pq] = T1[pr] * V[qr]", dpp, {{"A", A}, {"T1", T1}, {"V", V}});
  // B~ part: (W_perp B) V diag(1/f) V^T
  mm(ctx, "T3[nq] = B[np] * V[pq]", dnp, {{"T3", T3}, {"B", Bp}, {"V", V}});
  scale_cols(ctx, T3, g, n, p);
  mm(ctx, "Xo[nq] = T3[np] * V[qp]", dnp, {{"Xo", Xout.data}, {"T3", T3}, {"V", V}});
  mm(ctx, "Xo[nq] += W[np] * A[pq]", dnp, {{"Xo", Xout.data}, {"W", W.data}, {"A", A}});
}

void precondition_many(Ctx& ctx, const std::vector<MatView>& W, const std::vector<MatView>& X, Metric& met,
                       const std::vector<double>& delta, const std::vector<MatView>& Xout) {
  // factors of equal shape share grouped launches; each factor computes what precondition_one computes for it
  const size_t k = W.size();
  std::vector<bool> done(k, false);
  for (size_t a = 0; a < k; ++a) {
    if (done[a]) continue;
    std::vector<size_t> grp;
    for (size_t b = a; b < k && grp.size() < (size_t)kGettMaxGroup; ++b)
      if (!done[b] && W[b].n == W[a].n && W[b].p == W[a].p) {
        grp.push_back(b);
        done[b] = true;
      }
    const int n = W[a].n, p = W[a].p;
    const int64_t pp = (int64_t)p * p;
    const size_t G = grp.size();
    std::vector<double*> A(G), T1(G), Ah(G), Bp(G), T3(G), V(G), f(G), g(G);
    for (size_t j = 0; j < G; ++j) {
      const size_t i = grp[j];
      MERA_CHECK(met.p[i] == p, MERA_EINVAL, "metric size does not match the tensor");
      const std::string t = std::to_string(j);
      A[j] = tmp(ctx, "pc.A" + t, pp);
      T1[j] = tmp(ctx, "pc.T1" + t, pp);
      Ah[j] = tmp(ctx, "pc.Ah" + t, pp);
      Bp[j] = tmp(ctx, "pc.B" + t, (int64_t)n * p);
      T3[j] = tmp(ctx, "pc.T3" + t, (int64_t)n * p);
      V[j] = met.V[i].as<double>();
      f[j] = met.f[i].as<double>();
      g[j] = met.g[i].as<double>();
      reg_spectrum(ctx, met.lam[i].as<double>(), delta[i], f[j], g[j], p);
    }
    const std::initializer_list<std::pair<char, int64_t>> dpp = {{'p', p}, {'q', p}, {'r', p}};
    const std::initializer_list<std::pair<char, int64_t>> dnp = {{'n', n}, {'p', p}, {'q', p}};
    // A = W^T X; X = W A + (X - W A) with (X - W A) = W_perp B
    {
      std::vector<std::vector<void*>> s1(G), s2(G);
      for (size_t j = 0; j < G; ++j) {
        const size_t i = grp[j];
        s1[j] = {A[j], W[i].data, X[i].data};
        s2[j] = {Bp[j], W[i].data, A[j]};
      }
      mm_group(ctx, "A[pq] = W[np] * X[nq]", dnp, {"A", "W", "X"}, s1);
      for (size_t j = 0; j < G; ++j) copy(ctx, VPtr{Bp[j], Prec::F64}, d64(X[grp[j]]), (int64_t)n * p);
      mm_group(ctx, "B[nq] += -1.0 * W[np] * A[pq]", dnp, {"B", "W", "A"}, s2);
    }
    // A~ = V [ (V^T A V)_ij 2 / (f_i + f_j) ] V^T
    {
      std::vector<std::vector<void*>> s1(G), s2(G), s3(G), s4(G);
      for (size_t j = 0; j < G; ++j) {
        s1[j] = {T1[j], V[j], A[j]};
        s2[j] = {Ah[j], T1[j], V[j]};
        s3[j] = {T1[j], V[j], Ah[j]};
        s4[j] = {A[j], T1[j], V[j]};
      }
      mm_group(ctx, "T1[pq] = V[rp] * A[rq]", dpp, {"T1", "V", "A"}, s1);
      mm_group(ctx, "Ah[pq] = T1[pr] * V[rq]", dpp, {"Ah", "T1", "V"}, s2);
      for (size_t j = 0; j < G; ++j) scale_sylvester(ctx, Ah[j], f[j], p);
      mm_group(ctx, "T1[pq] = V[pr] * Ah[rq]", dpp, {"T1", "V", "Ah"}, s3);
      mm_group(ctx, "A[pq] = T1[pr] * V[qr]", dpp, {"A", "T1", "V"}, s4);
    }
    // B~ part: (W_perp B) V diag(1/f) V^T
    {
      std::vector<std::vector<void*>> s1(G), s2(G), s3(G);
      for (size_t j = 0; j < G; ++j) {
        const size_t i = grp[j];
        s1[j] = {T3[j], Bp[j], V[j]};
        s2[j] = {Xout[i].data, T3[j], V[j]};
        s3[j] = {Xout[i].data, W[i].data, A[j]};
      }
      mm_group(ctx, "T3[nq] = B[np] * V[pq]", dnp, {"T3", "B", "V"}, s1);
      for (size_t j = 0; j < G; ++j) scale_cols(ctx, T3[j], g[j], n, p);
      mm_group(ctx, "Xo[nq] = T3[np] * V[qp]", dnp, {"Xo", "T3", "V"}, s2);
      mm_group(ctx, "Xo[nq] += W[np] * A[pq]", dnp, {"Xo", "W", "A"}, s3);
    }
  }
}

// ---- L-BFGS ------------------------------------------------------------------------------------------

void Lbfgs::init(Ctx& ctx, const std::vector<int>& n, const std::vector<int>& p, int m_) {
  (void)ctx;
  MERA_CHECK(m_ >= 0, MERA_EINVAL, "L-BFGS memory must be >= 0");
  m = m_;
  shape.init(n, p);
  S.clear();
  Y.clear();
  for (int i = 0; i < m; ++i) {
    S.emplace_back((size_t)shape.total * 8);
    Y.emplace_back((size_t)shape.total * 8);
  }
  r.assign(m, 0.0);
  order.clear();
  q.alloc((size_t)shape.total * 8);
  z.alloc((size_t)shape.total * 8);
  t.alloc((size_t)shape.total * 8);
}

namespace {

std::vector<MatView> views_of(const Flat& shape, double* base) {
  std::vector<MatView> v;
  for (int i = 0; i < shape.count(); ++i) v.push_back(MatView{shape.n[i], shape.p[i], base + shape.off[i]});
  return v;
}

void gather(Ctx& ctx, const Flat& shape, const std::vector<MatView>& src, double* dst) {
  for (int i = 0; i < shape.count(); ++i)
    copy(ctx, VPtr{dst + shape.off[i], Prec::F64}, d64(src[i]), (int64_t)shape.n[i] * shape.p[i]);
}

void scatter(Ctx& ctx, const Flat& shape, const double* src, const std::vector<MatView>& dst, double scale) {
  for (int i = 0; i < shape.count(); ++i) {
    const int64_t k = (int64_t)shape.n[i] * shape.p[i];
    copy(ctx, d64(dst[i]), VPtr{(void*)(src + shape.off[i]), Prec::F64}, k);
    if (scale != 1.0) scal(ctx, scale, d64(dst[i]), k);
  }
}

void apply_precond(Ctx& ctx, const Flat& shape, const std::vector<MatView>& W, Metric* met, double* x,
                   double* out) {
  if (!met || met->empty()) {
    if (out != x) copy(ctx, VPtr{out, Prec::F64}, VPtr{x, Prec::F64}, shape.total);
    return;
  }
  auto xv = views_of(shape, x), ov = views_of(shape, out);
  // every factor's regularisation delta = |X_i| with one synchronisation
  const int nf = shape.count();
  std::vector<VPtr> xp(nf);
  std::vector<int64_t> ne(nf);
  std::vector<double> delta(nf);
  for (int i = 0; i < nf; ++i) {
    xp[i] = d64(xv[i]);
    ne[i] = numel(xv[i]);
  }
  dots(ctx, xp.data(), xp.data(), ne.data(), nf, delta.data());
  for (double& d : delta) d = std::sqrt(d);
  precondition_many(ctx, W, xv, *met, delta, ov);
}

}  // namespace

double Lbfgs::step(Ctx& ctx, const std::vector<MatView>& W, const std::vector<MatView>& G, Metric* met,
                   const std::vector<MatView>& dout) {
  const int64_t N = shape.total;
  double* qp = q.as<double>();
  double* zp = z.as<double>();
  double* tp = t.as<double>();
  VPtr Q{qp, Prec::F64}, Z{zp, Prec::F64}, Tt{tp, Prec::F64};
  gather(ctx, shape, G, qp);
  // The inner products stay on the device (one slot each: <s_k, q> and <y_k, z> of every pair, and the two of the
  // initial scaling), and every coefficient is formed there exactly as on the host (r <s_k, q>, then
  // r <s_k, q> - r <y_k, z>): the two loops need no host synchronisation.
  const size_t np = order.size();
  double* dsc = static_cast<double*>(ctx.buf("lb.scalars", (2 * np + 2) * sizeof(double)));
  double* dS = dsc;           // <s_k, q>
  double* dY = dsc + np;      // <y_k, z>
  double* dG = dsc + 2 * np;  // <s, y>, <y, H0 y> of the newest pair
  for (int k = (int)np - 1; k >= 0; --k) {
    const int sl = order[k];
    dot_dev_exact(ctx, S[sl].as<double>(), qp, N, dS + k);
    axpby_dev(ctx, dS + k, -r[sl], VPtr{Y[sl].ptr, Prec::F64}, 1.0, Q, N);  // q -= (r <s_k, q>) y_k
  }
  apply_precond(ctx, shape, W, met, qp, zp);
  if (!order.empty()) {
    const int sl = order.back();
    apply_precond(ctx, shape, W, met, Y[sl].as<double>(), tp);
    dot_dev_exact(ctx, S[sl].as<double>(), Y[sl].as<double>(), N, dG);
    dot_dev_exact(ctx, Y[sl].as<double>(), tp, N, dG + 1);
    scal_ratio_dev(ctx, dG, dG + 1, zp, N);  // z *= <s, y> / <y, H0 y>
  }
  for (size_t k = 0; k < np; ++k) {
    const int sl = order[k];
    dot_dev_exact(ctx, Y[sl].as<double>(), zp, N, dY + k);
    axpby_diff_dev(ctx, r[sl], dS + k, dY + k, S[sl].as<double>(), 1.0, zp, N);  // z += (alpha_k - beta_k) s_k
  }
  // d = -z
  gather(ctx, shape, G, tp);
  double slope = -dot(ctx, Tt, Z, N);
  if (!(slope < 0.0)) {
    order.clear();
    apply_precond(ctx, shape, W, met, tp, zp);
    slope = -dot(ctx, Tt, Z, N);
  }
  MERA_CHECK(std::isfinite(slope), MERA_ENONFINITE, "non-finite L-BFGS direction");
  scatter(ctx, shape, zp, dout, -1.0);
  return slope;
}

bool Lbfgs::push(Ctx& ctx, const std::vector<MatView>& Wn, const std::vector<MatView>& d, double alpha,
                 const std::vector<MatView>& Gold, const std::vector<MatView>& Gnew) {
  const Transport T = [&](int i, const MatView& in, const MatView& out) { stiefel_project_one(ctx, Wn[i], in, out); };
  const TransportMany TM = [&](const std::vector<int>& fac, const std::vector<MatView>& in,
                               const std::vector<MatView>& out) {
    std::vector<MatView> w;
    for (int i : fac) w.push_back(Wn[i]);
    project_many(ctx, w, in, out, std::vector<bool>(fac.size(), false));
  };
  return push(ctx, T, d, alpha, Gold, Gnew, TM);
}

bool Lbfgs::push(Ctx& ctx, const Transport& T, const std::vector<MatView>& d, double alpha,
                 const std::vector<MatView>& Gold, const std::vector<MatView>& Gnew, const TransportMany& TM) {
  const int64_t N = shape.total;
  // transport the stored pairs to the new point (all at once when TM is given)
  std::vector<int> fac;
  std::vector<MatView> items;
  for (int sl : order) {
    auto sv = views_of(shape, S[sl].as<double>()), yv = views_of(shape, Y[sl].as<double>());
    for (int i = 0; i < shape.count(); ++i) {
      if (TM) {
        fac.push_back(i);
        items.push_back(sv[i]);
        fac.push_back(i);
        items.push_back(yv[i]);
      } else {
        T(i, sv[i], sv[i]);
        T(i, yv[i], yv[i]);
      }
    }
  }
  if (TM && !items.empty()) TM(fac, items, items);
  if (m == 0) return false;
  // candidate slot: a free one, or the oldest
  int slot;
  if ((int)order.size() < m) {
    std::vector<bool> used(m, false);
    for (int sl : order) used[sl] = true;
    slot = 0;
    while (used[slot]) ++slot;
  } else {
    slot = order.front();
  }
  double* sp = q.as<double>();  // build in scratch first; the oldest pair stays valid if rejected
  double* yp = t.as<double>();
  auto sv = views_of(shape, sp), yv = views_of(shape, yp);
  for (int i = 0; i < shape.count(); ++i) {
    const int64_t k = (int64_t)shape.n[i] * shape.p[i];
    copy(ctx, d64(sv[i]), d64(d[i]), k);
    scal(ctx, alpha, d64(sv[i]), k);
    T(i, sv[i], sv[i]);
    T(i, Gold[i], yv[i]);
    axpby(ctx, 1.0, d64(Gnew[i]), -1.0, d64(yv[i]), k);
  }
  const double sy = dot(ctx, VPtr{sp, Prec::F64}, VPtr{yp, Prec::F64}, N);
  const double ss = dot(ctx, VPtr{sp, Prec::F64}, VPtr{sp, Prec::F64}, N);
  const double yy = dot(ctx, VPtr{yp, Prec::F64}, VPtr{yp, Prec::F64}, N);
  if (!(sy > 1e-12 * std::sqrt(ss * yy))) return false;
  copy(ctx, VPtr{S[slot].ptr, Prec::F64}, VPtr{sp, Prec::F64}, N);
  copy(ctx, VPtr{Y[slot].ptr, Prec::F64}, VPtr{yp, Prec::F64}, N);
  r[slot] = 1.0 / sy;
  if ((int)order.size() == m) order.erase(order.begin());
  order.push_back(slot);
  return true;
}

// ---- optimiser ----------------------------------------------------------------------------------------

JobSpec JobSpec::from_c(const mera_job& j) {
  JobSpec s;
  s.shape = j.shape;
  auto dims = layer_dims(j.shape);
  const int64_t hsize = dims[0].opsize(j.shape.d);  // d^6 (three-site, binary) or d^4 (two-site, ternary)
  MERA_CHECK(j.h3_host != nullptr, MERA_EINVAL, "job: null h3");
  MERA_CHECK(j.init_host != nullptr, MERA_EINVAL, "job: null initial tensors");
  s.h3.assign(j.h3_host, j.h3_host + (size_t)hsize);
  for (int t = 0; t <= j.shape.T; ++t) {
    const int a2 = dims[t].a * dims[t].a;
    const double* u = j.init_host[2 * t];
    const double* w = j.init_host[2 * t + 1];
    MERA_CHECK(u && w, MERA_EINVAL, "job: null initial tensor");
    s.init.emplace_back(u, u + (size_t)a2 * a2);
    s.init.emplace_back(w, w + (size_t)dims[t].wrows() * dims[t].b);
  }
  MERA_CHECK(j.prec == MERA_FP64 || j.prec == MERA_FP32 || j.prec == MERA_BF16X3, MERA_EINVAL, "job: precision");
  s.prec = j.prec == MERA_FP64 ? Prec::F64 : (j.prec == MERA_FP32 ? Prec::F32 : Prec::BF16X3);
  s.m = j.lbfgs_m;
  s.max_iter = j.max_iter;
  s.grad_tol = j.grad_tol;
  s.polish_tol = j.polish_tol;
  s.precondition = j.precondition != 0;
  s.max_ls_evals = j.max_ls_evals > 0 ? j.max_ls_evals : 10;
  MERA_CHECK(j.method >= 0 && j.method <= 2, MERA_EINVAL, "job: method must be 0 (L-BFGS), 1 (CG) or 2 (EV)");
  s.method = j.method;
  MERA_CHECK(j.method != 2 || (std::isfinite(j.ev_gamma) && j.ev_gamma > 0.0), MERA_EINVAL,
             "job: Evenbly-Vidal needs a positive ev_gamma");
  s.ev_gamma = j.ev_gamma;
  MERA_CHECK(j.retraction == 0 || j.retraction == 1, MERA_EINVAL, "job: retraction must be 0 (polar) or 1 (exp)");
  s.retraction = j.retraction;
  s.grassmann_w = j.grassmann_w != 0;
  if (j.krylov.krylov_dim > 0) s.krylov.dim = j.krylov.krylov_dim;
  if (j.krylov.max_restarts > 0) s.krylov.max_restarts = j.krylov.max_restarts;
  if (j.krylov.tol > 0) s.krylov.tol = j.krylov.tol;
  if (j.krylov.extrapolate != 0) s.krylov.extrapolate = j.krylov.extrapolate > 0;
  MERA_CHECK(s.m >= 0 && s.max_iter >= 0, MERA_EINVAL, "job: negative memory or iteration cap");
  return s;
}

void Optimizer::start(Ctx& c, const JobSpec& j, int log_cap_) {
  ctx = &c;
  job = j;
  log_cap = log_cap_;
  dims = layer_dims(job.shape);
  std::vector<int> n, p, rp;
  for (const LayerDim& L : dims) {
    n.push_back(L.a * L.a);
    p.push_back(L.a * L.a);
    n.push_back((int)L.wrows());
    p.push_back(L.b);
    rp.push_back(L.a * L.a);
    rp.push_back(L.b);
  }
  for (Flat* F : {&W, &G, &Wn, &Gn, &D, &Xp, &dir}) F->init(n, p);
  rv.init(rp, rp);
  rvn.init(rp, rp);
  hist.init(c, n, p, job.method == 0 ? job.m : 0);
  if (job.method == 1)
    for (Flat* F : {&cg_d, &cg_y, &cg_pg, &cg_py}) F->init(n, p);
  cg_have = false;
  grass.assign(n.size(), 0);
  for (size_t i = 1; i < n.size(); i += 2) grass[i] = job.grassmann_w ? 1 : 0;
  frames.clear();
  frames.resize(job.retraction == 1 ? n.size() : 0);
  const size_t h3n = job.h3.size();
  h3dev.alloc(h3n * 8);
  MERA_HIP(hipMemcpyAsync(h3dev.ptr, job.h3.data(), h3n * 8, hipMemcpyHostToDevice, c.stream));
  for (int i = 0; i < W.count(); ++i)
    MERA_HIP(hipMemcpyAsync(W.view(i).data, job.init[i].data(), job.init[i].size() * 8, hipMemcpyHostToDevice,
                            c.stream));
  prec = job.prec;
  macs0 = c.macs;
  iter = 0;
  evals = 0;
  done = false;
  started = true;
  result = OptResult();
  f = evaluate(W, G, rv);
  if (job.precondition) met.compute(c, rv.views());
}

double Optimizer::evaluate(const Flat& X, Flat& Gout, Flat& rvout) {
  Point pt;
  GradOut go;
  for (int t = 0; t < (int)dims.size(); ++t) {
    pt.u.push_back(X.view(2 * t).data);
    pt.w.push_back(X.view(2 * t + 1).data);
    go.Du.push_back(D.view(2 * t).data);
    go.Dw.push_back(D.view(2 * t + 1).data);
    if (need_rv()) {
      go.rho_u.push_back(rvout.view(2 * t).data);
      go.rho_w.push_back(rvout.view(2 * t + 1).data);
    }
  }
  EvalOut r = energy_grad(*ctx, job.shape, pt, h3dev.as<double>(), prec, &warm, job.krylov, go);
  evals++;
  krylov_apps += r.app_rho + r.app_ht;
  {
    std::vector<MatView> w, dv, gv;
    std::vector<bool> gr;
    for (int i = 0; i < X.count(); ++i) {
      w.push_back(X.view(i));
      dv.push_back(D.view(i));
      gv.push_back(Gout.view(i));
      gr.push_back(grass[i] != 0);
    }
    project_many(*ctx, w, dv, gv, gr);
  }
  return r.energy;
}

void Optimizer::project_factor(int i, const MatView& Wv, const MatView& Dv, const MatView& Gv) {
  if (grass[i]) grassmann_project_one(*ctx, Wv, Dv, Gv);
  else stiefel_project_one(*ctx, Wv, Dv, Gv);
}

void Optimizer::build_frames() {
  for (int i = 0; i < W.count(); ++i) exp_frame_one(*ctx, W.view(i), dir.view(i), frames[i]);
}

void Optimizer::transport_factor(int i, const MatView& in, const MatView& out) {
  if (job.retraction == 1) exp_apply_one(*ctx, W.view(i), frames[i], in, out);
  else project_factor(i, Wn.view(i), in, out);
}

bool Optimizer::advance() {
  if (done) return true;
  Ctx& c = *ctx;
  gnorm = std::sqrt(inner(c, G.views(), G.views()));
  MERA_CHECK(std::isfinite(gnorm), MERA_ENONFINITE, "non-finite gradient norm");
  if ((int)result.log.size() < log_cap)
    result.log.push_back(mera_iter_log{iter, evals, f, gnorm, last_alpha, (int)prec});
  if (gnorm <= job.grad_tol) {
    status = 0;
    done = true;
    return true;
  }
  if (iter >= job.max_iter) {
    status = 1;
    done = true;
    return true;
  }
  // precision switch: below the polishing threshold the contractions move to FP64 and the point is re-evaluated
  if (prec != Prec::F64 && job.polish_tol > 0 && gnorm < job.polish_tol) {
    prec = Prec::F64;
    polish_iter = iter;
    f = evaluate(W, G, rv);
    if (job.precondition) met.compute(c, rv.views());
    return false;  // the iteration restarts from the re-evaluated point
  }
  if (job.method == 2) {
    ev_sweep();
    return false;
  }
  Metric* mp = job.precondition ? &met : nullptr;
  const auto Wv = W.views();
  const bool cg = job.method == 1;
  bool momentum = false;
  double alpha0 = 1.0;
  double slope = cg ? cg_direction(mp, momentum, alpha0) : hist.step(c, Wv, G.views(), mp, dir.views());
  const bool expr = job.retraction == 1;
  if (expr) build_frames();

  double f_trial = 0.0;
  auto phi = [&](double alpha, double& fa, double& dfa) {
    if (expr) {
      for (int i = 0; i < W.count(); ++i) {
        MatView xo = Xp.view(i);
        exp_retract_one(c, W.view(i), dir.view(i), frames[i], alpha, Wn.view(i), &xo);
      }
    } else {
      const std::vector<MatView> xo = Xp.views();
      std::vector<const MatView*> xop(xo.size());
      for (size_t i = 0; i < xo.size(); ++i) xop[i] = &xo[i];
      stiefel_retract_many(c, W.views(), dir.views(), alpha, Wn.views(), xop);
    }
    fa = evaluate(Wn, Gn, rvn);
    dfa = inner(c, Gn.views(), Xp.views());
    f_trial = fa;
  };
  // Wolfe / approximate-Wolfe line search (same rules as the reference optimiser of the tests)
  auto line_search = [&](double f0, double df0, double a0, double& alpha_out) {
    const double c1 = 1e-4, c2 = 0.9, eps = 1e-6;
    const double epsk = eps * std::fabs(f0);
    double lo_a = 0.0, lo_df = df0;
    double hi_a = std::numeric_limits<double>::infinity();
    double hi_df = std::numeric_limits<double>::quiet_NaN();
    bool has_hi_df = false;
    double alpha = a0;
    for (int k = 1; k <= job.max_ls_evals; ++k) {
      double fa, dfa;
      phi(alpha, fa, dfa);
      if (!(std::isfinite(fa) && std::isfinite(dfa))) {
        hi_a = alpha;
        hi_df = std::numeric_limits<double>::infinity();
        has_hi_df = true;
      } else {
        const bool wolfe = fa <= f0 + c1 * alpha * df0 && dfa >= c2 * df0;
        const bool approx = (2.0 * c1 - 1.0) * df0 >= dfa && dfa >= c2 * df0 && fa <= f0 + epsk;
        if (wolfe || approx) {
          alpha_out = alpha;
          return true;
        }
        if (dfa >= 0.0 || fa > f0 + epsk) {
          hi_a = alpha;
          hi_df = dfa;
          has_hi_df = true;
        } else {
          lo_a = alpha;
          lo_df = dfa;
        }
      }
      if (std::isinf(hi_a)) {
        alpha = 2.0 * alpha;
        continue;
      }
      const double width = hi_a - lo_a;
      double trial = std::numeric_limits<double>::quiet_NaN();
      if (has_hi_df && std::isfinite(hi_df) && hi_df >= 0.0 && hi_df > lo_df)
        trial = (lo_a * hi_df - hi_a * lo_df) / (hi_df - lo_df);
      if (!(lo_a + 0.1 * width <= trial && trial <= hi_a - 0.1 * width)) trial = lo_a + 0.5 * width;
      alpha = trial;
    }
    return false;
  };
  double alpha = 0.0;
  bool ok = line_search(f, slope, alpha0, alpha);
  if (!ok && !cg && hist.size() > 0) {
    hist.reset();
    slope = hist.step(c, Wv, G.views(), mp, dir.views());
    if (expr) build_frames();
    ok = line_search(f, slope, 1.0, alpha);
  } else if (!ok && cg && momentum) {
    cg_restart(mp);
    slope = inner(c, G.views(), dir.views());
    if (expr) build_frames();
    ok = line_search(f, slope, 1.0, alpha);
  }
  if (!ok && prec != Prec::F64 && job.polish_tol > 0) {
    // Near the noise floor of the reduced-precision energy the expected decrease of a step falls below the
    // energy's rounding error and the Wolfe conditions can no longer be met: polishing starts here instead,
    // from the current point re-evaluated in FP64, with the history dropped (its pairs came from the noisy
    // gradients).
    prec = Prec::F64;
    polish_iter = iter;
    hist.reset();
    cg_have = false;
    f = evaluate(W, G, rv);
    if (job.precondition) met.compute(c, rv.views());
    return false;
  }
  if (!ok) {
    status = 2;
    done = true;
    return true;
  }
  // Wn, Gn, rvn hold the accepted (last evaluated) point
  // exponential transport uses E of the accepted alpha, the last one evaluated
  const Lbfgs::Transport T = [&](int i, const MatView& in, const MatView& out) { transport_factor(i, in, out); };
  if (cg) {
    // previous direction and gradient carried to the new point by the transport; y = G_new - T(G_old)
    for (int i = 0; i < W.count(); ++i) {
      T(i, dir.view(i), cg_d.view(i));
      T(i, G.view(i), cg_y.view(i));
    }
    axpby(c, 1.0, VPtr{Gn.ptr(), Prec::F64}, -1.0, VPtr{cg_y.ptr(), Prec::F64}, cg_y.total);
    cg_gold = gnorm;
    cg_alpha_prev = alpha;
    cg_slope_prev = slope;
    cg_have = true;
  } else {
    const Lbfgs::TransportMany TM = [&](const std::vector<int>& fac, const std::vector<MatView>& in,
                                        const std::vector<MatView>& out) {
      if (job.retraction == 1) {
        for (size_t j = 0; j < fac.size(); ++j) transport_factor(fac[j], in[j], out[j]);
        return;
      }
      std::vector<MatView> w;
      std::vector<bool> gr;
      for (int i : fac) {
        w.push_back(Wn.view(i));
        gr.push_back(grass[i]);
      }
      project_many(c, w, in, out, gr);
    };
    hist.push(c, T, dir.views(), alpha, G.views(), Gn.views(), TM);
  }
  std::swap(W.buf, Wn.buf);
  std::swap(G.buf, Gn.buf);
  std::swap(rv.buf, rvn.buf);
  f = f_trial;
  last_alpha = alpha;
  iter++;
  if (job.precondition) met.compute(c, rv.views());
  return false;
}

void Optimizer::ev_sweep() {
  Ctx& c = *ctx;
  // u_1, w_1, ..., u_s, w_s in turn, each from a fresh environment (the first reuses the current evaluation)
  for (int i = 0; i < W.count(); ++i) {
    if (i > 0) f = evaluate(W, G, rv);
    ev_update_one(c, W.view(i), D.view(i), rv.view(i), job.ev_gamma, Wn.view(i));
    copy(c, d64(W.view(i)), d64(Wn.view(i)), (int64_t)W.view(i).n * W.view(i).p);
  }
  f = evaluate(W, G, rv);
  if (job.precondition) met.compute(c, rv.views());
  last_alpha = 0.0;
  iter++;
}

void Optimizer::cg_restart(Metric* met) {
  Ctx& c = *ctx;
  apply_precond(c, G, W.views(), met, G.ptr(), cg_pg.ptr());
  copy(c, VPtr{dir.ptr(), Prec::F64}, VPtr{cg_pg.ptr(), Prec::F64}, G.total);
  scal(c, -1.0, VPtr{dir.ptr(), Prec::F64}, G.total);
}

double Optimizer::cg_direction(Metric* met, bool& momentum, double& alpha0) {
  Ctx& c = *ctx;
  const int64_t N = G.total;
  const VPtr g{G.ptr(), Prec::F64}, pg{cg_pg.ptr(), Prec::F64}, d{dir.ptr(), Prec::F64};
  const VPtr pd{cg_d.ptr(), Prec::F64}, y{cg_y.ptr(), Prec::F64}, py{cg_py.ptr(), Prec::F64};
  cg_restart(met);  // dir = -P G (and cg_pg = P G)
  momentum = false;
  if (cg_have) {
    apply_precond(c, G, W.views(), met, cg_y.ptr(), cg_py.ptr());
    const double dy = dot(c, pd, y, N);
    double beta = 0.0;
    if (dy != 0.0 && std::isfinite(dy)) {
      // preconditioned Hager-Zhang coefficient, truncated below as in Hager and Zhang
      beta = dot(c, y, pg, N) / dy - 2.0 * dot(c, y, py, N) * dot(c, pd, g, N) / (dy * dy);
      const double dn = std::sqrt(dot(c, pd, pd, N));
      if (dn > 0.0 && cg_gold > 0.0) beta = std::max(beta, -1.0 / (dn * std::min(0.01, cg_gold)));
    }
    axpby(c, beta, pd, 1.0, d, N);
    momentum = true;
  }
  double slope = dot(c, g, d, N);
  if (!(slope < 0.0)) {
    cg_restart(met);
    slope = dot(c, g, d, N);
    momentum = false;
  }
  alpha0 = (momentum && cg_alpha_prev > 0.0) ? cg_alpha_prev * cg_slope_prev / slope : 1.0;
  return slope;
}

void Optimizer::finish(std::vector<double*>* final_host) {
  Ctx& c = *ctx;
  if (final_host && !final_host->empty()) {
    MERA_CHECK((int)final_host->size() == W.count(), MERA_EINVAL, "final tensor count");
    for (int i = 0; i < W.count(); ++i)
      if ((*final_host)[i])
        MERA_HIP(hipMemcpyAsync((*final_host)[i], W.view(i).data, (size_t)numel(W.view(i)) * 8,
                                hipMemcpyDeviceToHost, c.stream));
  }
  c.sync();
  result.energy = f;
  result.gnorm = std::sqrt(inner(c, G.views(), G.views()));
  result.iterations = iter;
  result.evaluations = evals;
  result.status = status;
  result.polish_iter = polish_iter;
  result.krylov_apps = krylov_apps;
  result.macs = c.macs - macs0;
}

size_t Optimizer::device_bytes() const {
  size_t b = 0;
  for (const Flat* F : {&W, &G, &Wn, &Gn, &D, &Xp, &dir, &rv, &rvn, &cg_d, &cg_y, &cg_pg, &cg_py}) b += F->buf.bytes;
  b += warm.rho.bytes + warm.ht.bytes + h3dev.bytes;
  for (auto& x : hist.S) b += x.bytes;
  for (auto& x : hist.Y) b += x.bytes;
  return b;
}

OptResult optimize(Ctx& ctx, const JobSpec& job, std::vector<double*>* final_host, int log_cap) {
  const auto t0 = std::chrono::steady_clock::now();
  Optimizer opt;
  opt.start(ctx, job, log_cap);
  while (!opt.advance()) {
  }
  opt.finish(final_host);
  opt.result.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return opt.result;
}

}  // namespace mera
