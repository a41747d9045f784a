// Host planner of the H-LU library.
//
//  * cluster tree (Algorithm 1 of the paper, Sec. 2): tight axis-parallel
//    boxes, split of the longest axis at the box midpoint, median split if
//    one side would be empty;
//  * block tree (Algorithm 2) with min(diam t, diam s) <= eta * dist(t, s);
//  * host assembly: near-field blocks exactly, far-field blocks by adaptive
//    cross approximation followed by Householder QR of both factors and a
//    Jacobi SVD of the small core (the "SVD recompression" of Sec. 6.1),
//    truncated once for the factor copy and once for the refinement copy;
//  * a static schedule: the recursive H-LU (Sec. 3.1 sequence O1.1-O5.5 and
//    the partitioned solves O2.1-O2.6 of Sec. 5.2) is walked once and every
//    primitive operation becomes a descriptor; a descriptor's wave is one
//    more than the latest wave it conflicts with (read/write sets tracked per
//    leaf cluster of every panel), the device analogue of the paper's
//    skeleton array of representants (Secs. 4.1 and 5.1).
#include "plan.hpp"

#include <algorithm>
#include <map>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <thread>

namespace hlu {

static const double kFourPi = 4.0 * M_PI;

// ---------------------------------------------------------------- entries
// Collocation entries between panel midpoints x_i with one-point quadrature
// over the column panel (weight a_j: area, or length for the 1D and 2D
// kernels) plus the identity.  Kernels (Sec. 6.1): 1/(4 pi r) (d = 3),
// -log r (d = 1), -log(r) / (2 pi) (d = 2).  The self term of a d = 1 or
// d = 2 panel is the exact integral of the kernel over the straight panel
// of length h around its midpoint: h (1 - log(h / 2)), times 1 / (2 pi) for
// d = 2.
struct Entries {
  const double* x;
  const double* a;
  int kernel;
  // doubled plans: positions [0, n1) and [n1, 2 n1) are two copies of the
  // same points; each quadrant holds 0, A (kernel), B (kernel_b) or I
  int n1 = 0, op = 0, kernel_b = 0;
  inline double operator()(int i, int j) const {
    if (op == 0) return base(kernel, i, j);
    const int qi = i >= n1, qj = j >= n1, ii = i - qi * n1, jj = j - qj * n1;
    if (op == 1) {
      if (qi == 0 && qj == 1) return base(kernel, ii, jj);
      if (qi == 1 && qj == 0) return base(kernel_b, ii, jj);
      return 0.0;
    }
    if (qi == 0 && qj == 0) return base(kernel, ii, jj);
    if (qi != qj) return ii == jj ? 1.0 : 0.0;
    return 0.0;
  }
  inline double base(int kernel, int i, int j) const {
    if (i == j) {
      if (kernel == 2) return a[i] * (1.0 - std::log(0.5 * a[i])) + 1.0;
      if (kernel == 3) return a[i] * (1.0 - std::log(0.5 * a[i])) / (2.0 * M_PI) + 1.0;
      return 2.0 * std::sqrt(a[i] / M_PI) / kFourPi * std::sqrt(M_PI) + 1.0;
    }
    double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1],
           dz = x[3 * i + 2] - x[3 * j + 2];
    double r = std::sqrt(dx * dx + dy * dy + dz * dz);
    if (kernel == 2) return -a[j] * std::log(r);
    if (kernel == 3) return -a[j] * std::log(r) / (2.0 * M_PI);
    double g = 1.0 / (kFourPi * r);
    return kernel == 0 ? g * a[j] : g;
  }
};

// ---------------------------------------------------------------- trees
static int build_cluster(Plan& p, std::vector<int>& idx, int lo_i, int hi_i,
                         const double* X, std::vector<int64_t>& order) {
  int id = (int)p.cl.size();
  p.cl.emplace_back();
  Cluster c;
  c.size = hi_i - lo_i;
  for (int d = 0; d < 3; ++d) { c.lo[d] = INFINITY; c.hi[d] = -INFINITY; }
  for (int k = lo_i; k < hi_i; ++k)
    for (int d = 0; d < 3; ++d) {
      double v = X[3 * idx[k] + d];
      c.lo[d] = std::min(c.lo[d], v);
      c.hi[d] = std::max(c.hi[d], v);
    }
  if (c.size > p.prm.leaf) {
    int d = 0;
    for (int e = 1; e < 3; ++e)
      if (c.hi[e] - c.lo[e] > c.hi[d] - c.lo[d]) d = e;
    double mid = 0.5 * (c.lo[d] + c.hi[d]);
    std::vector<int> a, b;
    for (int k = lo_i; k < hi_i; ++k) (X[3 * idx[k] + d] < mid ? a : b).push_back(idx[k]);
    if (a.empty() || b.empty()) {
      std::vector<int> s(idx.begin() + lo_i, idx.begin() + hi_i);
      std::stable_sort(s.begin(), s.end(), [&](int u, int v) {
        double xu = X[3 * u + d], xv = X[3 * v + d];
        return xu < xv || (xu == xv && u < v);
      });
      a.assign(s.begin(), s.begin() + c.size / 2);
      b.assign(s.begin() + c.size / 2, s.end());
    }
    int na = (int)a.size();
    std::copy(a.begin(), a.end(), idx.begin() + lo_i);
    std::copy(b.begin(), b.end(), idx.begin() + lo_i + na);
    p.cl[id] = c;
    int s0 = build_cluster(p, idx, lo_i, lo_i + na, X, order);
    int s1 = build_cluster(p, idx, lo_i + na, hi_i, X, order);
    p.cl[id].son[0] = s0;
    p.cl[id].son[1] = s1;
    p.cl[id].off = p.cl[s0].off;
    p.cl[id].first_leaf = p.cl[s0].first_leaf;
    p.cl[id].nleaves = p.cl[s0].nleaves + p.cl[s1].nleaves;
  } else {
    c.off = (int)order.size();
    c.leaf = (int)p.leaves.size();
    c.first_leaf = c.leaf;
    c.nleaves = 1;
    for (int k = lo_i; k < hi_i; ++k) order.push_back(idx[k]);
    p.cl[id] = c;
    p.leaves.push_back(id);
  }
  return id;
}

static bool admissible(const Cluster& t, const Cluster& s, double eta) {
  double g2 = 0.0, dt2 = 0.0, ds2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    double g = std::max(0.0, std::max(s.lo[d] - t.hi[d], t.lo[d] - s.hi[d]));
    g2 += g * g;
    dt2 += (t.hi[d] - t.lo[d]) * (t.hi[d] - t.lo[d]);
    ds2 += (s.hi[d] - s.lo[d]) * (s.hi[d] - s.lo[d]);
  }
  double dist = std::sqrt(g2);
  if (eta <= 0.0 || dist <= 0.0) return false;
  return std::min(std::sqrt(dt2), std::sqrt(ds2)) <= eta * dist;
}

static int build_blocks(Plan& p, int t, int s) {
  int id = (int)p.bn.size();
  p.bn.push_back(BNode{t, s, 'F'});
  const Cluster &ct = p.cl[t], &cs = p.cl[s];
  if (admissible(ct, cs, p.prm.eta)) {
    p.bn[id].kind = 'R';
  } else if (ct.son[0] >= 0 && cs.son[0] >= 0) {
    p.bn[id].kind = 'H';
    int k = 0;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        int c = build_blocks(p, ct.son[i], cs.son[j]);
        p.bn[id].son[k++] = c;
      }
    return id;
  }
  LBlock b;
  b.t = t;
  b.s = s;
  b.kind = p.bn[id].kind;
  b.m = ct.size;
  b.n = cs.size;
  p.bn[id].blk = (int)p.blk.size();
  p.blk.push_back(b);
  return id;
}

// ---------------------------------------------------------------- small dense LA (host)
// Householder QR of A (m x k, column-major, ld m) in place; reflectors below
// the diagonal, tau[min(m,k)].
static void house_qr(double* A, int m, int k, std::vector<double>& tau) {
  int r = std::min(m, k);
  tau.assign(r, 0.0);
  for (int j = 0; j < r; ++j) {
    double* x = A + j + (size_t)j * m;
    int len = m - j;
    double nrm = 0.0;
    for (int i = 1; i < len; ++i) nrm += x[i] * x[i];
    double alpha = x[0];
    if (nrm == 0.0) { tau[j] = 0.0; continue; }
    double beta = -std::copysign(std::sqrt(alpha * alpha + nrm), alpha);
    tau[j] = (beta - alpha) / beta;
    double sc = 1.0 / (alpha - beta);
    for (int i = 1; i < len; ++i) x[i] *= sc;
    x[0] = beta;
    for (int c = j + 1; c < k; ++c) {
      double* y = A + j + (size_t)c * m;
      double w = y[0];
      for (int i = 1; i < len; ++i) w += x[i] * y[i];
      w *= tau[j];
      y[0] -= w;
      for (int i = 1; i < len; ++i) y[i] -= w * x[i];
    }
  }
}

// B (m x c, ld m) := Q B with Q from house_qr (B's rows >= r are inputs too).
static void apply_q(const double* A, int m, int k, const std::vector<double>& tau, double* B,
                    int c) {
  int r = std::min(m, k);
  for (int j = r - 1; j >= 0; --j) {
    if (tau[j] == 0.0) continue;
    const double* x = A + j + (size_t)j * m;
    int len = m - j;
    for (int q = 0; q < c; ++q) {
      double* y = B + j + (size_t)q * m;
      double w = y[0];
      for (int i = 1; i < len; ++i) w += x[i] * y[i];
      w *= tau[j];
      y[0] -= w;
      for (int i = 1; i < len; ++i) y[i] -= w * x[i];
    }
  }
}

// One-sided Jacobi SVD of M (r1 x r2, ld r1): M = W diag(sig) Z^T with
// sig sorted descending; W: r1 x r2, Z: r2 x r2.
static void jacobi_svd(std::vector<double> M, int r1, int r2, std::vector<double>& W,
                       std::vector<double>& sig, std::vector<double>& Z) {
  std::vector<double> V((size_t)r2 * r2, 0.0);
  for (int i = 0; i < r2; ++i) V[i + (size_t)i * r2] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rot = false;
    for (int a = 0; a < r2 - 1; ++a)
      for (int b = a + 1; b < r2; ++b) {
        double al = 0, be = 0, ga = 0;
        double* ca = &M[(size_t)a * r1];
        double* cb = &M[(size_t)b * r1];
        for (int i = 0; i < r1; ++i) {
          al += ca[i] * ca[i];
          be += cb[i] * cb[i];
          ga += ca[i] * cb[i];
        }
        if (std::fabs(ga) <= 1e-15 * std::sqrt(al * be) || ga == 0.0) continue;
        rot = true;
        double zeta = (be - al) / (2.0 * ga);
        double t = std::copysign(1.0, zeta) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < r1; ++i) {
          double x = ca[i], y = cb[i];
          ca[i] = c * x - s * y;
          cb[i] = s * x + c * y;
        }
        double* va = &V[(size_t)a * r2];
        double* vb = &V[(size_t)b * r2];
        for (int i = 0; i < r2; ++i) {
          double x = va[i], y = vb[i];
          va[i] = c * x - s * y;
          vb[i] = s * x + c * y;
        }
      }
    if (!rot) break;
  }
  std::vector<double> nrm(r2);
  for (int j = 0; j < r2; ++j) {
    double s = 0;
    for (int i = 0; i < r1; ++i) s += M[i + (size_t)j * r1] * M[i + (size_t)j * r1];
    nrm[j] = std::sqrt(s);
  }
  std::vector<int> ord(r2);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int u, int v) { return nrm[u] > nrm[v]; });
  W.assign((size_t)r1 * r2, 0.0);
  Z.assign((size_t)r2 * r2, 0.0);
  sig.assign(r2, 0.0);
  for (int jj = 0; jj < r2; ++jj) {
    int j = ord[jj];
    sig[jj] = nrm[j];
    for (int i = 0; i < r1; ++i)
      W[i + (size_t)jj * r1] = nrm[j] > 0 ? M[i + (size_t)j * r1] / nrm[j] : 0.0;
    for (int i = 0; i < r2; ++i) Z[i + (size_t)jj * r2] = V[i + (size_t)j * r2];
  }
}

// Rank choice: fixed, or smallest k with ||sig_{k:}|| <= eps ||sig||, capped.
static int choose_rank(const std::vector<double>& sig, double eps, int cap, int fixed,
                       bool* capped) {
  int r = (int)sig.size();
  *capped = false;
  if (fixed > 0) return std::min(fixed, r);
  double tot = 0;
  for (double s : sig) tot += s * s;
  double thr = eps * eps * tot;
  double tail = 0;
  int k = r;
  // tail over indices >= k, growing from the end
  for (int j = r; j >= 0; --j) {
    if (tail <= thr) k = j;
    else break;
    if (j > 0) tail += sig[j - 1] * sig[j - 1];
  }
  if (k > cap) { *capped = true; k = cap; }
  return k;
}

// Adaptive cross approximation with partial pivoting of the m x n block
// starting at (r0, c0); returns U (m x k), V (n x k) with block ~= U V^T.
static void aca(const Entries& E, int r0, int c0, int m, int n, double eps, int kmax,
                std::vector<double>& U, std::vector<double>& V, int& k) {
  U.clear();
  V.clear();
  k = 0;
  std::vector<char> urow(m, 0), ucol(n, 0);
  std::vector<double> row(n), col(m);
  double norm2 = 0.0;
  int i = 0, small = 0, zero_tries = 0;
  while (k < kmax) {
    for (int j = 0; j < n; ++j) {
      double v = E(r0 + i, c0 + j);
      for (int l = 0; l < k; ++l) v -= U[i + (size_t)l * m] * V[j + (size_t)l * n];
      row[j] = v;
    }
    urow[i] = 1;
    int js = -1;
    double best = 0.0;
    for (int j = 0; j < n; ++j)
      if (!ucol[j] && std::fabs(row[j]) > best) { best = std::fabs(row[j]); js = j; }
    if (js < 0 || best == 0.0) {
      // zero residual row: try another unused row
      int nx = -1;
      for (int q = 0; q < m; ++q)
        if (!urow[q]) { nx = q; break; }
      if (nx < 0 || ++zero_tries > 3) break;
      i = nx;
      continue;
    }
    ucol[js] = 1;
    double piv = row[js];
    for (int q = 0; q < m; ++q) {
      double v = E(r0 + q, c0 + js);
      for (int l = 0; l < k; ++l) v -= V[js + (size_t)l * n] * U[q + (size_t)l * m];
      col[q] = v;
    }
    U.resize((size_t)(k + 1) * m);
    V.resize((size_t)(k + 1) * n);
    double nu = 0, nv = 0;
    for (int q = 0; q < m; ++q) { U[q + (size_t)k * m] = col[q]; nu += col[q] * col[q]; }
    for (int j = 0; j < n; ++j) { V[j + (size_t)k * n] = row[j] / piv; nv += (row[j] / piv) * (row[j] / piv); }
    double cross = 0.0;
    for (int l = 0; l < k; ++l) {
      double a = 0, b = 0;
      for (int q = 0; q < m; ++q) a += U[q + (size_t)l * m] * U[q + (size_t)k * m];
      for (int j = 0; j < n; ++j) b += V[j + (size_t)l * n] * V[j + (size_t)k * n];
      cross += a * b;
    }
    norm2 += nu * nv + 2.0 * cross;
    ++k;
    if (std::sqrt(nu * nv) <= eps * std::sqrt(std::fabs(norm2))) {
      if (++small >= 2) break;
    } else {
      small = 0;
    }
    int inext = -1;
    best = -1.0;
    for (int q = 0; q < m; ++q)
      if (!urow[q] && std::fabs(col[q]) > best) { best = std::fabs(col[q]); inext = q; }
    if (inext < 0) break;
    i = inext;
  }
}

// Recompress U V^T (ranks ka) by QR + SVD; return the singular triplets as
// Uk = Q_U W Sigma, Vk = Q_V Z (all r columns, sorted).
static void recompress(std::vector<double>& U, std::vector<double>& V, int m, int n, int ka,
                       std::vector<double>& sig, std::vector<double>& Uo,
                       std::vector<double>& Vo, int& r) {
  std::vector<double> tu, tv;
  house_qr(U.data(), m, ka, tu);
  house_qr(V.data(), n, ka, tv);
  int r1 = std::min(m, ka), r2 = std::min(n, ka);
  // M = R_U R_V^T  (r1 x r2)
  std::vector<double> M((size_t)r1 * r2, 0.0);
  for (int i = 0; i < r1; ++i)
    for (int j = 0; j < r2; ++j) {
      double s = 0;
      for (int l = std::max(i, j); l < ka; ++l) s += U[i + (size_t)l * m] * V[j + (size_t)l * n];
      M[i + (size_t)j * r1] = s;
    }
  std::vector<double> W, Z;
  jacobi_svd(M, r1, r2, W, sig, Z);
  r = std::min(r1, r2);
  sig.resize(r);
  Uo.assign((size_t)m * r, 0.0);
  Vo.assign((size_t)n * r, 0.0);
  for (int j = 0; j < r; ++j) {
    for (int i = 0; i < r1; ++i) Uo[i + (size_t)j * m] = W[i + (size_t)j * r1] * sig[j];
    for (int i = 0; i < r2; ++i) Vo[i + (size_t)j * n] = Z[i + (size_t)j * r2];
  }
  apply_q(U.data(), m, ka, tu, Uo.data(), r);
  apply_q(V.data(), n, ka, tv, Vo.data(), r);
}

template <class F>
static void parallel_for(int count, F&& f) {
  unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        int i = next.fetch_add(1);
        if (i >= count) break;
        f(i);
      }
    });
  for (auto& x : th) x.join();
}

// ---------------------------------------------------------------- schedule builder
namespace {

struct Obj {
  int first_leaf = 0, nleaves = 1;
  bool whole_only = false;
  std::vector<int> W, R;
  int wW = -1, wR = -1, mW = -1, mR = -1;
};

struct PV {                  // planner-side panel view
  int obj = -1;
  uint64_t off = 0;          // byte offset
  int ld = 0, rows = 0, cols = 0;
  uint64_t rank = 0;         // byte offset of the dynamic column count (0: static)
  int dt = DT_F64;
  int trans = 0, ident = 0;
  int cl = -1;               // cluster of the rows
  int robj = -1;             // object written whenever the dynamic count changes
  int diag = 0;              // identity: element (i, j) is 1 iff j == i + diag
};

struct Acc {
  int obj;
  int l0, l1;                // global leaf range; l0 < 0: whole object
  bool write;
};

class Builder {
 public:
  Builder(Plan& p, Schedule& s) : P(p), S(s) {}
  Plan& P;
  Schedule& S;
  std::vector<Obj> objs;
  std::vector<Op> ops;
  std::vector<int> wave;
  uint64_t scratch_cur = 0, scratch_base = 0;
  uint64_t cost_cur = 0;
  bool want_cost = true;
  int P_dt = DT_F64;
  int chunk_cols = 32;

  int new_obj(int cl, bool whole_only) {
    Obj o;
    if (cl >= 0) {
      o.first_leaf = P.cl[cl].first_leaf;
      o.nleaves = P.cl[cl].nleaves;
    }
    o.whole_only = whole_only || cl < 0;
    if (!o.whole_only) {
      o.W.assign(o.nleaves, -1);
      o.R.assign(o.nleaves, -1);
    }
    objs.push_back(std::move(o));
    return (int)objs.size() - 1;
  }

  Acc racc(const PV& v) { return Acc{v.robj, -1, -1, false}; }
  Acc acc_of(const PV& v, bool write) {
    if (v.obj < 0) return Acc{-1, -1, -1, write};
    const Obj& o = objs[v.obj];
    if (o.whole_only || v.cl < 0) return Acc{v.obj, -1, -1, write};
    const Cluster& c = P.cl[v.cl];
    return Acc{v.obj, c.first_leaf, c.first_leaf + c.nleaves, write};
  }
  Acc whole(int obj, bool write) { return Acc{obj, -1, -1, write}; }

  int schedule(const std::vector<Acc>& acc) {
    int dep = extra_wave;
    extra_wave = -1;
    for (const Acc& a : acc) {
      if (a.obj < 0) continue;
      Obj& o = objs[a.obj];
      if (a.l0 < 0) {
        dep = std::max(dep, o.mW);
        if (a.write) dep = std::max(dep, o.mR);
      } else {
        dep = std::max(dep, o.wW);
        if (a.write) dep = std::max(dep, o.wR);
        for (int l = a.l0; l < a.l1; ++l) {
          int q = l - o.first_leaf;
          dep = std::max(dep, o.W[q]);
          if (a.write) dep = std::max(dep, o.R[q]);
        }
      }
    }
    int w = dep + 1;
    for (const Acc& a : acc) {
      if (a.obj < 0) continue;
      Obj& o = objs[a.obj];
      if (a.l0 < 0) {
        if (a.write) { o.wW = std::max(o.wW, w); o.mW = std::max(o.mW, w); }
        else { o.wR = std::max(o.wR, w); o.mR = std::max(o.mR, w); }
      } else {
        for (int l = a.l0; l < a.l1; ++l) {
          int q = l - o.first_leaf;
          if (a.write) o.W[q] = std::max(o.W[q], w);
          else o.R[q] = std::max(o.R[q], w);
        }
        if (a.write) o.mW = std::max(o.mW, w);
        else o.mR = std::max(o.mR, w);
      }
    }
    return w;
  }

  PRef ref(const PV& v) {
    PRef r;
    std::memset(&r, 0, sizeof(r));
    r.ptr = v.off;
    r.rankp = v.rank;
    r.ld = v.ld;
    r.rows = v.rows;
    r.cols = v.cols;
    r.dt = (uint8_t)v.dt;
    r.trans = (uint8_t)v.trans;
    r.kind = v.ident ? PK_IDENT : PK_MAT;
    if (v.ident) { r.ld = v.diag; r.ptr = 0; }
    return r;
  }

  // ---- exact dependency edges (for the dataflow executor): per object part
  // the last writer and the readers since; an op depends on the last writer
  // of every part it touches and, when it writes, on the readers since.
  struct EObj {
    int first_leaf = 0, nparts = 1;
    std::vector<int> lastW;
    std::vector<std::vector<int>> readers;
  };
  std::vector<EObj> eobjs;
  std::vector<std::vector<int>> preds;       // emission order
  bool want_edges = true;

  void eobj_sync() {
    while (eobjs.size() < objs.size()) {
      const Obj& o = objs[eobjs.size()];
      EObj e;
      e.first_leaf = o.first_leaf;
      e.nparts = o.whole_only ? 1 : o.nleaves;
      e.lastW.assign(e.nparts, -1);
      e.readers.resize(e.nparts);
      eobjs.push_back(std::move(e));
    }
  }

  void edges(const std::vector<Acc>& acc, int self) {
    eobj_sync();
    std::vector<int> pr;
    pr.swap(extra_pred);
    auto range = [&](const Acc& a, int& p0, int& p1) {
      const EObj& o = eobjs[a.obj];
      if (a.l0 < 0 || o.nparts == 1) { p0 = 0; p1 = o.nparts; }
      else { p0 = a.l0 - o.first_leaf; p1 = a.l1 - o.first_leaf; }
    };
    for (const Acc& a : acc) {
      if (a.obj < 0) continue;
      int p0, p1;
      range(a, p0, p1);
      EObj& o = eobjs[a.obj];
      for (int p = p0; p < p1; ++p) {
        if (o.lastW[p] >= 0) pr.push_back(o.lastW[p]);
        if (a.write) pr.insert(pr.end(), o.readers[p].begin(), o.readers[p].end());
      }
    }
    for (const Acc& a : acc) {
      if (a.obj < 0 || a.write) continue;
      int p0, p1;
      range(a, p0, p1);
      EObj& o = eobjs[a.obj];
      for (int p = p0; p < p1; ++p) o.readers[p].push_back(self);
    }
    for (const Acc& a : acc) {
      if (a.obj < 0 || !a.write) continue;
      int p0, p1;
      range(a, p0, p1);
      EObj& o = eobjs[a.obj];
      for (int p = p0; p < p1; ++p) {
        o.lastW[p] = self;
        o.readers[p].clear();
      }
    }
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    if (!pr.empty() && pr.back() == self) pr.pop_back();
    preds.push_back(std::move(pr));
  }

  void emit(Op op, const std::vector<Acc>& acc) {
    int w = schedule(acc);
    if (want_edges) edges(acc, (int)ops.size());
    if (want_cost) {
      op.cost = cost_cur;
      cost_cur += kCostRecBytes;
    } else {
      op.cost = 0;
    }
    ops.push_back(op);
    wave.push_back(w);
  }

  static Op blank(int type) {
    Op o;
    std::memset(&o, 0, sizeof(o));
    o.type = type;
    return o;
  }

  // ---- panel helpers
  PV sub(const PV& v, int child) {     // rows restricted to a child cluster
    PV r = v;
    const Cluster& c = P.cl[child];
    const Cluster& pc = P.cl[v.cl];
    int d = c.off - pc.off;
    if (v.ident) {
      r.diag = v.diag + d;
      r.rows = c.size;
      r.cl = child;
      return r;
    }
    int es = v.dt == DT_F64 ? 8 : 4;
    r.off = v.off + (uint64_t)(v.trans ? (uint64_t)d * v.ld : (uint64_t)d) * es;
    r.rows = c.size;
    r.cl = child;
    return r;
  }
  PV row_range(const PV& v, int r0, int nrows) {   // rows r0 .. r0 + nrows - 1
    PV r = v;
    const int es = v.dt == DT_F64 ? 8 : 4;
    r.off = v.off + (uint64_t)(v.trans ? (uint64_t)r0 * v.ld : (uint64_t)r0) * es;
    r.rows = nrows;
    r.cl = -1;
    return r;
  }
  PV dense_panel(int b) {             // F block as panel over its rows
    const LBlock& B = P.blk[b];
    PV v;
    v.obj = B.objF;
    v.off = B.offF;
    v.ld = B.m;
    v.rows = B.m;
    v.cols = B.n;
    v.cl = B.t;
    v.dt = DT_F64;
    return v;
  }
  PV dense_panelT(int b) {            // transpose of an F block (rows = columns)
    const LBlock& B = P.blk[b];
    PV v;
    v.obj = B.objF;
    v.off = B.offF;
    v.ld = B.m;
    v.rows = B.n;
    v.cols = B.m;
    v.cl = B.s;
    v.trans = 1;
    v.dt = DT_F64;
    return v;
  }
  PV u_panel(int b) {
    const LBlock& B = P.blk[b];
    PV v;
    v.obj = B.objU;
    v.off = B.offU;
    v.ld = B.m;
    v.rows = B.m;
    v.cols = P.prm.cap_f;
    v.rank = B.offRank;
    v.robj = B.objRank;
    v.cl = B.t;
    v.dt = P_dt;
    return v;
  }
  PV v_panel(int b) {
    const LBlock& B = P.blk[b];
    PV v;
    v.obj = B.objV;
    v.off = B.offV;
    v.ld = B.n;
    v.rows = B.n;
    v.cols = P.prm.cap_f;
    v.rank = B.offRank;
    v.robj = B.objRank;
    v.cl = B.s;
    v.dt = P_dt;
    return v;
  }
  PV ident(int cl) {
    PV v;
    v.ident = 1;
    v.diag = 0;
    v.rows = P.cl[cl].size;
    v.cols = P.cl[cl].size;
    v.cl = cl;
    v.dt = DT_F64;
    return v;
  }
  // ---- reuse of the scratch region as a ring (when ring_cap > 0).  Live
  // allocations are kept by address.  A new allocation evicts every tenant it
  // overlaps and takes over the whole extent of each (so no byte a retired
  // tenant touched is ever free without a successor that orders after its
  // ops); its first op (the zeroing) then depends on every op that touched
  // them.  At a wrap the tail tenants stay live until the ring reaches them
  // again.  Tenants still referenced by deferred truncation terms are
  // consumed (flushed) first.
  struct Live {
    uint64_t off, end;
    int obj;
  };
  std::map<uint64_t, Live> live;    // keyed by off
  uint64_t ring_cap = 0, ring_cur = 0;
  int extra_wave = -1;              // lower bound for the next op's wave
  std::vector<int> extra_pred;      // extra predecessors of the next op
  std::vector<char> pend_obj;       // object referenced by a pending term
  void retire(int obj) {
    const Obj& o = objs[obj];
    extra_wave = std::max(extra_wave, std::max(o.mW, o.mR));
    if (!want_edges) return;
    eobj_sync();
    const EObj& e = eobjs[obj];
    for (int q = 0; q < e.nparts; ++q) {
      if (e.lastW[q] >= 0) extra_pred.push_back(e.lastW[q]);
      extra_pred.insert(extra_pred.end(), e.readers[q].begin(), e.readers[q].end());
    }
  }
  bool is_pending(int obj) const { return obj >= 0 && obj < (int)pend_obj.size() && pend_obj[obj]; }
  std::map<uint64_t, Live>::iterator first_overlap(uint64_t off) {
    auto it = live.upper_bound(off);
    if (it != live.begin()) {
      auto p = std::prev(it);
      if (p->second.end > off) return p;
    }
    return it;
  }
  // Returns the data offset of a new allocation of `bytes`; `ext` receives
  // the extent the new tenant owns (the data plus absorbed evicted ranges).
  uint64_t ring_alloc(uint64_t bytes, Live& ext) {
    if (bytes > ring_cap) {
      P.err = "scratch_cap_bytes is smaller than one H-GEMM temporary (" + std::to_string(bytes) +
              " bytes)";
      ext = Live{0, 0, -1};
      return 0;
    }
    const uint64_t off = ring_cur + bytes > ring_cap ? 0 : ring_cur;
    uint64_t lo = off, hi = off + bytes;
    bool flush = false;
    for (auto it = first_overlap(off); it != live.end() && it->first < hi; ++it)
      flush |= is_pending(it->second.obj);
    if (flush) flush_truncations();
    for (auto it = first_overlap(off); it != live.end() && it->first < hi;) {
      lo = std::min(lo, it->second.off);
      hi = std::max(hi, it->second.end);
      retire(it->second.obj);
      it = live.erase(it);
    }
    ring_cur = hi;
    scratch_cur = std::max(scratch_cur, hi);
    ext = Live{lo, hi, -1};
    return off;
  }

  PV scratch(int cl, int cols, uint64_t rank, int dt, int robj = -1) {
    PV v;
    v.robj = robj;
    int es = dt == DT_F64 ? 8 : 4;
    uint64_t bytes = (uint64_t)P.cl[cl].size * cols * es;
    bytes = (bytes + 255) & ~(uint64_t)255;
    if (ring_cap > 0) {
      Live ext;
      const uint64_t off = ring_alloc(bytes, ext);
      v.obj = new_obj(cl, false);
      ext.obj = v.obj;
      live[ext.off] = ext;
      v.off = scratch_base + off;
    } else {
      v.obj = new_obj(cl, false);
      v.off = scratch_base + scratch_cur;
      scratch_cur += bytes;
    }
    v.ld = P.cl[cl].size;
    v.rows = P.cl[cl].size;
    v.cols = cols;
    v.rank = rank;
    v.cl = cl;
    v.dt = dt;
    if (ring_cap > 0) {
      // zero it (static capacity columns); in a ring the zeroing op also
      // orders the new tenant after every op that touched the extent
      Op z = blank(OP_ZERO);
      PV zz = v;
      zz.rank = 0;
      z.p[0] = ref(zz);
      emit(z, {acc_of(v, true)});
    } else {
      // fresh memory: the first product into each row range overwrites it
      // (every scratch panel is filled by one panel product over its row
      // cluster right after its allocation; consumers read live columns only)
      if ((int)fresh_rows.size() <= v.obj) fresh_rows.resize(v.obj + 1);
      fresh_rows[v.obj].clear();
      fresh_rows[v.obj].push_back(-1);   // marker: tracked, nothing written yet
    }
    return v;
  }
  // per fresh scratch object: [lo, hi) row ranges written so far (first
  // entry -1 marks a tracked object)
  std::vector<std::vector<int64_t>> fresh_rows;
  // true iff rows [lo, hi) of object obj are tracked and untouched; marks them
  bool first_write(int obj, int64_t lo, int64_t hi) {
    if (obj < 0 || obj >= (int)fresh_rows.size() || fresh_rows[obj].empty()) return false;
    std::vector<int64_t>& w = fresh_rows[obj];
    for (size_t q = 1; q + 1 < w.size(); q += 2)
      if (lo < w[q + 1] && w[q] < hi) return false;
    w.push_back(lo);
    w.push_back(hi);
    return true;
  }

  const BNode& node(int b) const { return P.bn[b]; }
  int son(int b, int i, int j) const { return P.bn[b].son[2 * i + j]; }

  // ---- primitive emitters
  void getrf(int nb) {
    const LBlock& B = P.blk[node(nb).blk];
    Op op = blank(OP_GETRF);
    op.p[0] = ref(dense_panel(node(nb).blk));
    op.p[1].ptr = P.off_piv + (uint64_t)P.cl[B.t].off * 4;
    op.p[1].rankp = P.off_status;
    op.i0 = P.cl[B.t].off;
    emit(op, {whole(B.objF, true)});
    // the leaf's inverses for the solve (read by no factor op)
    Op inv = blank(OP_TRINV);
    inv.p[0] = op.p[0];
    inv.p[1].ptr = op.p[1].ptr;
    inv.p[2] = inv_ref(P.off_inv_l, B.t);
    inv.p[3] = inv_ref(P.off_inv_u, B.t);
    emit(inv, {whole(B.objF, false)});
  }
  PRef inv_ref(uint64_t region, int cl) const {
    PRef r;
    std::memset(&r, 0, sizeof(r));
    const int b = P.cl[cl].size;
    r.ptr = region + (uint64_t)P.cl[cl].off * 64 * 8;
    r.ld = b;
    r.rows = b;
    r.cols = b;
    r.dt = DT_F64;
    r.kind = PK_MAT;
    return r;
  }
  // solve: Y := W Y with the precomputed inverse W of the leaf of nb.  When
  // a row update on exactly these rows was the last op to write them (no op
  // reads them before the leaf is solved), the product is fused into that
  // op (i2 = 1, W in p0), one op and one hand-off less on the sweep's chain.
  void inv_apply(uint64_t region, int nb, const PV& Y) {
    const LBlock& L = P.blk[node(nb).blk];
    if ((int)last_row_op.size() > L.t && last_row_op[L.t] >= 0) {
      Op& u = ops[last_row_op[L.t]];
      last_row_op[L.t] = -1;
      const PRef yr = ref(Y);
      if (u.type == OP_MVROW && u.p[3].ptr == yr.ptr && u.p[3].rows == yr.rows &&
          u.p[3].ld == yr.ld) {
        u.p[0] = inv_ref(region, L.t);
        u.i2 = 1;
        return;
      }
    }
    Op op = blank(OP_INVAPPLY);
    op.p[0] = inv_ref(region, L.t);
    op.p[1] = ref(Y);
    emit(op, {acc_of(Y, true), racc(Y)});
  }
  void trsm_leaf(int type, int nb, const PV& Y) {
    const LBlock& L = P.blk[node(nb).blk];
    Op op = blank(type);
    op.p[0] = ref(dense_panel(node(nb).blk));
    op.p[1] = ref(Y);
    op.p[2].ptr = P.off_piv + (uint64_t)P.cl[L.t].off * 4;
    emit(op, {whole(L.objF, false), acc_of(Y, true), racc(Y)});
  }
  // Y += sign * op(M) X, M any block node
  void pmul(const PV& Y, int nb, const PV& X, double sign, bool tr) {
    const BNode& M = node(nb);
    if (M.kind == 'H') {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          int c = son(nb, i, j);
          const BNode& C = node(c);
          if (!tr) pmul(sub(Y, C.t), c, sub(X, C.s), sign, tr);
          else pmul(sub(Y, C.s), c, sub(X, C.t), sign, tr);
        }
      return;
    }
    const LBlock& B = P.blk[M.blk];
    Op op = blank(OP_PGEMM);
    op.d0 = sign;
    op.i1 = tr ? 1 : 0;
    {
      // rows of Y this product writes (Y is restricted to this block's
      // row cluster, or its column cluster when transposed)
      const Cluster& rc = P.cl[Y.cl];
      const int64_t lo = (int64_t)rc.off, hi = lo + rc.size;
      if (first_write(Y.obj, lo, hi)) op.i2 = 1;
    }
    op.p[2] = ref(X);
    op.p[3] = ref(Y);
    std::vector<Acc> acc = {acc_of(X, false), acc_of(Y, true), racc(X), racc(Y)};
    if (M.kind == 'F') {
      op.i0 = 0;
      op.p[0] = ref(dense_panel(M.blk));
      acc.push_back(whole(B.objF, false));
    } else {
      op.i0 = 1;
      op.p[0] = ref(u_panel(M.blk));
      op.p[1] = ref(v_panel(M.blk));
      acc.push_back(whole(B.objU, false));
      acc.push_back(whole(B.objV, false));
      acc.push_back(whole(B.objRank, false));
    }
    emit(op, acc);
  }

  // ---- solve updates as an H-matvec: Y[rows of M] -= M X for a block node M
  // off the diagonal.  First T_b := V_b^T X[cols of b] for every low-rank leaf
  // block b of M (one op each, all independent); then, per leaf cluster r of
  // M's rows, the contributions U_b[r] T_b and F_b[r] X[cols of b] summed in
  // a fixed order by two ops: the first takes the blocks whose columns avoid
  // the column leaf the sweep solves last (ready before it, off the sweep's
  // chain), the second the blocks that touch it (usually one small block
  // next to the diagonal).
  bool solve_mv = false;
  std::vector<int> Tobj;     // per block: object of its V^T X slot
  // solve: per leaf cluster, the last emitted row-update op on its rows
  // (-1: none since the leaf's last inverse application)
  std::vector<int> last_row_op;
  void block_leaves(int nb, std::vector<int>& out) {
    if (node(nb).kind == 'H') {
      for (int i = 0; i < 4; ++i) block_leaves(P.bn[nb].son[i], out);
    } else {
      out.push_back(nb);
    }
  }
  void cluster_leaves(int c, std::vector<int>& out) {
    if (P.cl[c].son[0] < 0) {
      out.push_back(c);
      return;
    }
    cluster_leaves(P.cl[c].son[0], out);
    cluster_leaves(P.cl[c].son[1], out);
  }
  PV tslot(int b, int nrhs_cols) {
    const LBlock& B = P.blk[b];
    PV v;
    v.obj = Tobj[b];
    v.off = B.offT;
    v.ld = P.prm.cap_f;
    v.rows = P.prm.cap_f;
    v.cols = nrhs_cols;
    v.dt = DT_F64;
    return v;
  }
  void hupd(const PV& Y, int nb, const PV& X, bool backward) {
    if ((int)Tobj.size() < (int)P.blk.size()) Tobj.assign(P.blk.size(), -1);
    std::vector<int> lv;
    block_leaves(nb, lv);
    for (int bn : lv) {
      const BNode& M = node(bn);
      if (M.kind != 'R') continue;
      const LBlock& B = P.blk[M.blk];
      if (Tobj[M.blk] < 0) Tobj[M.blk] = new_obj(-1, true);
      PV Xs = sub(X, M.s);
      PV T = tslot(M.blk, X.cols);
      const Cluster& sc = P.cl[M.s];
      if (sc.nleaves == 1) {
        Op op = blank(OP_MVT);
        op.p[0] = ref(v_panel(M.blk));
        op.p[2] = ref(Xs);
        op.p[3] = ref(T);
        emit(op, {whole(B.objV, false), whole(B.objRank, false), acc_of(Xs, false), racc(Xs),
                  whole(T.obj, true)});
        continue;
      }
      // several leaves: the rows of all but the leaf this sweep solves last
      // first (ready before that leaf, off the sweep's chain), then that
      // leaf's rows accumulated (i2 = 1)
      const int ll = P.leaves[backward ? sc.first_leaf : sc.first_leaf + sc.nleaves - 1];
      const Cluster& lc = P.cl[ll];
      const int rest0 = backward ? lc.size : 0, nrest = sc.size - lc.size;
      PV V = v_panel(M.blk);
      const int rl0 = backward ? sc.first_leaf + 1 : sc.first_leaf;
      Acc xr = acc_of(Xs, false);
      if (xr.l0 >= 0) xr = Acc{Xs.obj, rl0, rl0 + sc.nleaves - 1, false};
      Op a = blank(OP_MVT);
      a.p[0] = ref(row_range(V, rest0, nrest));
      a.p[2] = ref(row_range(Xs, rest0, nrest));
      a.p[3] = ref(T);
      emit(a, {whole(B.objV, false), whole(B.objRank, false), xr, racc(Xs),
               whole(T.obj, true)});
      PV Xl = sub(Xs, ll);
      Op b = blank(OP_MVT);
      b.i2 = 1;
      b.p[0] = ref(sub(V, ll));
      b.p[2] = ref(Xl);
      b.p[3] = ref(T);
      emit(b, {whole(B.objV, false), whole(B.objRank, false), acc_of(Xl, false), racc(Xl),
               whole(T.obj, true)});
    }
    std::vector<int> rows;
    cluster_leaves(node(nb).t, rows);
    // the column leaf this sweep solves last among M's columns
    const Cluster& cc = P.cl[node(nb).s];
    const int last_leaf = backward ? cc.first_leaf : cc.first_leaf + cc.nleaves - 1;
    for (int r : rows) {
      const Cluster& rc = P.cl[r];
      PV Yr = sub(Y, r);
      for (int late = 0; late < 2; ++late) {
        Op op = blank(OP_MVROW);
        op.p[3] = ref(Yr);
        op.d0 = -1.0;
        op.i0 = (int)S.terms.size();
        std::vector<Acc> acc = {acc_of(Yr, true), racc(Yr)};
        for (int bn : lv) {
          const BNode& M = node(bn);
          const Cluster& tc = P.cl[M.t];
          if (rc.first_leaf < tc.first_leaf || rc.first_leaf >= tc.first_leaf + tc.nleaves)
            continue;
          const Cluster& sc = P.cl[M.s];
          const bool touches = last_leaf >= sc.first_leaf && last_leaf < sc.first_leaf + sc.nleaves;
          if (touches != (late == 1)) continue;
          const LBlock& B = P.blk[M.blk];
          Term t;
          std::memset(&t, 0, sizeof(t));
          if (M.kind == 'R') {
            t.X = ref(sub(u_panel(M.blk), r));
            t.Y = ref(tslot(M.blk, X.cols));
            acc.push_back(whole(B.objU, false));
            acc.push_back(whole(B.objRank, false));
            acc.push_back(whole(Tobj[M.blk], false));
            S.terms.push_back(t);
          } else {
            // a dense leaf may be wider than 64 (a leaf cluster against a
            // larger one): one term per window of at most 64 columns
            PV Xs = sub(X, M.s);
            PV Fr = sub(dense_panel(M.blk), r);
            for (int c0 = 0; c0 < B.n; c0 += 64) {
              const int w = std::min(64, B.n - c0);
              PV xw = Xs;
              xw.off = Xs.off + (uint64_t)c0 * 8;   // rows c0.. of the FP64 vector panel
              xw.rows = w;
              t.X = ref(colwin(Fr, c0, w));
              t.Y = ref(xw);
              S.terms.push_back(t);
            }
            acc.push_back(whole(B.objF, false));
            acc.push_back(acc_of(Xs, false));
          }
        }
        // at most 256 terms per op (the row kernel's table); longer lists
        // become several ops on the same rows, ordered by their writes
        const int tend = (int)S.terms.size();
        for (int t0 = op.i0; t0 < tend; t0 += 256) {
          Op o2 = op;
          o2.i0 = t0;
          o2.i1 = std::min(256, tend - t0);
          emit(o2, acc);
          // the last op writing this leaf row (the leaf's inverse may be
          // fused into it)
          if ((int)last_row_op.size() < (int)P.cl.size()) last_row_op.assign(P.cl.size(), -1);
          last_row_op[r] = (int)ops.size() - 1;
        }
      }
    }
  }

  // Y := L^{-1} P Y over the rows of diagonal node nb
  void fwd(int nb, const PV& Y) {
    if (node(nb).kind == 'F') {
      if (solve_mv) inv_apply(P.off_inv_l, nb, Y);
      else trsm_leaf(OP_TRSM_L, nb, Y);
      return;
    }
    const BNode& L = node(nb);
    int t0 = P.cl[L.t].son[0], t1 = P.cl[L.t].son[1];
    PV Y0 = sub(Y, t0), Y1 = sub(Y, t1);
    fwd(son(nb, 0, 0), Y0);
    if (solve_mv) hupd(Y1, son(nb, 1, 0), Y0, false);
    else pmul(Y1, son(nb, 1, 0), Y0, -1.0, false);
    fwd(son(nb, 1, 1), Y1);
  }
  // Y := U^{-T} Y
  void bwdT(int nb, const PV& Y) {
    if (node(nb).kind == 'F') { trsm_leaf(OP_TRSM_UT, nb, Y); return; }
    const BNode& U = node(nb);
    int t0 = P.cl[U.t].son[0], t1 = P.cl[U.t].son[1];
    PV Y0 = sub(Y, t0), Y1 = sub(Y, t1);
    bwdT(son(nb, 0, 0), Y0);
    pmul(Y1, son(nb, 0, 1), Y0, -1.0, true);
    bwdT(son(nb, 1, 1), Y1);
  }
  // Y := U^{-1} Y
  void bwd(int nb, const PV& Y) {
    if (node(nb).kind == 'F') {
      if (solve_mv) inv_apply(P.off_inv_u, nb, Y);
      else trsm_leaf(OP_TRSM_U, nb, Y);
      return;
    }
    const BNode& U = node(nb);
    int t0 = P.cl[U.t].son[0], t1 = P.cl[U.t].son[1];
    PV Y0 = sub(Y, t0), Y1 = sub(Y, t1);
    bwd(son(nb, 1, 1), Y1);
    if (solve_mv) hupd(Y0, son(nb, 0, 1), Y1, true);
    else pmul(Y0, son(nb, 0, 1), Y1, -1.0, false);
    bwd(son(nb, 0, 0), Y0);
  }

  void trsm_l(int Lb, int Bb) {
    const BNode& B = node(Bb);
    if (B.kind == 'R') fwd(Lb, u_panel(B.blk));
    else if (B.kind == 'F') fwd(Lb, dense_panel(B.blk));
    else {
      for (int j = 0; j < 2; ++j) trsm_l(son(Lb, 0, 0), son(Bb, 0, j));
      for (int j = 0; j < 2; ++j) gemm(son(Bb, 1, j), son(Lb, 1, 0), son(Bb, 0, j));
      for (int j = 0; j < 2; ++j) trsm_l(son(Lb, 1, 1), son(Bb, 1, j));
    }
  }
  void trsm_u(int Bb, int Ub) {
    const BNode& B = node(Bb);
    if (B.kind == 'R') bwdT(Ub, v_panel(B.blk));
    else if (B.kind == 'F') bwdT(Ub, dense_panelT(B.blk));
    else {
      for (int i = 0; i < 2; ++i) trsm_u(son(Bb, i, 0), son(Ub, 0, 0));
      for (int i = 0; i < 2; ++i) gemm(son(Bb, i, 1), son(Bb, i, 0), son(Ub, 0, 1));
      for (int i = 0; i < 2; ++i) trsm_u(son(Bb, i, 1), son(Ub, 1, 1));
    }
  }

  // C := C - X Y^T with X placed at row xo of C's rows, Y at row yo
  // (xo, yo are non-zero only for a low-rank C)
  void add(int Cb, const PV& X, const PV& Y, int xo, int yo) {
    const BNode& C = node(Cb);
    if (C.kind == 'H') {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          int c = son(Cb, i, j);
          add(c, sub(X, node(c).t), sub(Y, node(c).s), 0, 0);
        }
      return;
    }
    const LBlock& B = P.blk[C.blk];
    if (C.kind == 'F') {
      if (xo != 0 || yo != 0) P.err = "offset update of a dense block";
      Op op = blank(OP_ADDD);
      op.p[0] = ref(dense_panel(C.blk));
      op.p[1] = ref(X);
      op.p[2] = ref(Y);
      emit(op, {whole(B.objF, true), acc_of(X, false), acc_of(Y, false), racc(X), racc(Y)});
      return;
    }
    // low-rank target: a dynamic-rank term has at most cap columns; static
    // terms are split into windows of at most chunk_cols columns
    bool dyn = X.rank != 0 || Y.rank != 0;
    if (dyn) {
      trunc(Cb, X, Y, xo, yo, 0, -1);
      return;
    }
    int cols = X.cols;
    for (int c0 = 0; c0 < cols; c0 += chunk_cols) {
      int w = std::min(chunk_cols, cols - c0);
      trunc(Cb, X, Y, xo, yo, c0, cols <= chunk_cols ? -1 : w);
    }
  }

  // column window [c0, c0+w) of a term; w < 0: all columns
  PV colwin(const PV& v, int c0, int w) {
    if (w < 0) return v;
    PV r = v;
    if (v.ident) {
      r.diag = v.diag - c0;
      r.cols = w;
      return r;
    }
    int es = v.dt == DT_F64 ? 8 : 4;
    r.off = v.off + (uint64_t)(v.trans ? (uint64_t)c0 : (uint64_t)c0 * v.ld) * es;
    r.cols = w;
    return r;
  }

  // Terms for low-rank targets are collected during one H-GEMM call and
  // added by one truncation op per target at the end of the call (the
  // target is never an operand of its own call, so deferring is exact).
  struct PendTerm {
    PV X, Y;
    int xo, yo;
  };
  std::vector<int> pend_order;
  std::vector<std::vector<PendTerm>> pend;   // indexed by block node
  static constexpr int kMaxTermsPerOp = 16;

  void trunc(int Cb, const PV& X, const PV& Y, int xo, int yo, int c0, int w) {
    if (pend.size() < P.bn.size()) pend.resize(P.bn.size());
    if (pend[Cb].empty()) pend_order.push_back(Cb);
    pend[Cb].push_back(PendTerm{colwin(X, c0, w), colwin(Y, c0, w), xo, yo});
    for (int ob : {X.obj, Y.obj})
      if (ob >= 0) {
        if ((int)pend_obj.size() <= ob) pend_obj.resize(ob + 1, 0);
        pend_obj[ob] = 1;
      }
    trunc_groups.insert(((int64_t)call_id << 24) ^ Cb);
  }

  void flush_truncations() {
    for (int Cb : pend_order) {
      const BNode& C = node(Cb);
      const LBlock& B = P.blk[C.blk];
      std::vector<PendTerm>& L = pend[Cb];
      for (size_t t0 = 0; t0 < L.size(); t0 += kMaxTermsPerOp) {
        size_t t1 = std::min(L.size(), t0 + kMaxTermsPerOp);
        Op op = blank(OP_TRUNC);
        op.p[0] = ref(u_panel(C.blk));
        op.p[1] = ref(v_panel(C.blk));
        op.i0 = (int32_t)S.terms.size();
        op.i1 = (int32_t)(t1 - t0);
        op.i2 = P.prm.cap_f | (P.prm.fixed_rank << 16);
        op.d0 = P.prm.eps_f;
        std::vector<Acc> acc = {whole(B.objU, true), whole(B.objV, true),
                                whole(B.objRank, true)};
        for (size_t t = t0; t < t1; ++t) {
          Term tm;
          std::memset(&tm, 0, sizeof(tm));
          tm.X = ref(L[t].X);
          tm.Y = ref(L[t].Y);
          tm.xo = L[t].xo;
          tm.yo = L[t].yo;
          S.terms.push_back(tm);
          acc.push_back(acc_of(L[t].X, false));
          acc.push_back(acc_of(L[t].Y, false));
          acc.push_back(racc(L[t].X));
          acc.push_back(racc(L[t].Y));
        }
        emit(op, acc);
      }
      for (const PendTerm& t : L)
        for (int ob : {t.X.obj, t.Y.obj})
          if (ob >= 0 && ob < (int)pend_obj.size()) pend_obj[ob] = 0;
      L.clear();
    }
    pend_order.clear();
  }
  int64_t call_id = 0;
  std::set<int64_t> trunc_groups;

  // C := C - A B   (C at rows xo / columns yo of a low-rank ancestor when
  // lr_target >= 0)
  void gemm(int Cb, int Ab, int Bb) {
    ++call_id;
    gemm_at(Cb, Ab, Bb, 0, 0);
    flush_truncations();
  }

  void gemm_at(int Cb, int Ab, int Bb, int xo, int yo) {
    const BNode &C = node(Cb), &A = node(Ab), &B = node(Bb);
    if (A.kind == 'R') {
      PV AU = u_panel(A.blk);
      PV Z = scratch(B.s, P.prm.cap_f, AU.rank, P_dt, AU.robj);
      pmul(Z, Bb, v_panel(A.blk), 1.0, true);
      add(Cb, AU, Z, xo, yo);
    } else if (B.kind == 'R') {
      PV BU = u_panel(B.blk);
      PV Z = scratch(A.t, P.prm.cap_f, BU.rank, P_dt, BU.robj);
      pmul(Z, Ab, BU, 1.0, false);
      add(Cb, Z, v_panel(B.blk), xo, yo);
    } else if (A.kind == 'F' && B.kind == 'F') {
      if (P.cl[A.s].son[0] < 0) {
        add(Cb, dense_panel(A.blk), dense_panelT(B.blk), xo, yo);
      } else if (C.kind == 'F') {
        add(Cb, dense_panel(A.blk), dense_panelT(B.blk), xo, yo);
      } else {
        PV Z = scratch(A.t, P.cl[B.s].size, 0, DT_F64);
        pmul(Z, Ab, dense_panel(B.blk), 1.0, false);
        add(Cb, Z, ident(B.s), xo, yo);
      }
    } else if (A.kind == 'H' && B.kind == 'F') {
      PV Z = scratch(A.t, P.cl[B.s].size, 0, DT_F64);
      pmul(Z, Ab, dense_panel(B.blk), 1.0, false);
      add(Cb, Z, ident(B.s), xo, yo);
    } else if (A.kind == 'F' && B.kind == 'H') {
      PV Z = scratch(B.s, P.cl[A.t].size, 0, DT_F64);
      pmul(Z, Bb, dense_panelT(A.blk), 1.0, true);
      add(Cb, ident(A.t), Z, xo, yo);
    } else {
      if (C.kind == 'H') {
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            for (int l = 0; l < 2; ++l)
              gemm_at(son(Cb, i, j), son(Ab, i, l), son(Bb, l, j), 0, 0);
      } else if (C.kind == 'R') {
        // products of the sons added to the whole low-rank target, each
        // placed at its rows / columns (zero elsewhere)
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            for (int l = 0; l < 2; ++l) {
              int a = son(Ab, i, l), b = son(Bb, l, j);
              int dxo = P.cl[node(a).t].off - P.cl[A.t].off;
              int dyo = P.cl[node(b).s].off - P.cl[B.s].off;
              gemm_at(Cb, a, b, xo + dxo, yo + dyo);
            }
      } else {
        P.err = "dense target with two partitioned operands";
      }
    }
  }

  void lu(int nb) {
    const BNode& A = node(nb);
    if (A.kind == 'F') { getrf(nb); return; }
    lu(son(nb, 0, 0));
    trsm_l(son(nb, 0, 0), son(nb, 0, 1));
    trsm_u(son(nb, 1, 0), son(nb, 0, 0));
    gemm(son(nb, 1, 1), son(nb, 1, 0), son(nb, 0, 1));
    lu(son(nb, 1, 1));
  }

  void finish() {
    int n = (int)ops.size();
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
      if (wave[a] != wave[b]) return wave[a] < wave[b];
      return ops[a].type < ops[b].type;
    });
    S.ops.resize(n);
    S.batches.clear();
    S.waves_list.clear();
    S.waves = 0;
    for (int k = 0; k < n; ++k) {
      S.ops[k] = ops[idx[k]];
      // record slots follow the schedule order
      S.ops[k].cost = want_cost ? (uint64_t)k * kCostRecBytes : 0;
      int w = wave[idx[k]], t = ops[idx[k]].type;
      if (S.batches.empty() || S.batches.back().wave != w || S.batches.back().type != t)
        S.batches.push_back(Batch{w, t, k, 0, 1u << t});
      S.batches.back().count++;
      if (S.waves_list.empty() || S.waves_list.back().wave != w)
        S.waves_list.push_back(Batch{w, -1, k, 0, 0u});
      S.waves_list.back().count++;
      S.waves_list.back().mask |= 1u << t;
      S.waves = std::max(S.waves, w + 1);
    }
    // successor lists in schedule order
    S.succ_off.clear();
    S.succ.clear();
    S.indeg0.clear();
    S.ready0.clear();
    if (!want_edges) return;
    std::vector<int> pos(n);
    for (int k = 0; k < n; ++k) pos[idx[k]] = k;
    std::vector<int32_t> cnt(n + 1, 0);
    S.indeg0.assign(n, 0);
    for (int e = 0; e < n; ++e) {
      S.indeg0[pos[e]] = (int32_t)preds[e].size();
      for (int p : preds[e]) cnt[pos[p] + 1]++;
    }
    for (int k = 0; k < n; ++k) cnt[k + 1] += cnt[k];
    S.succ_off = cnt;
    S.succ.assign(cnt[n], 0);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int e = 0; e < n; ++e)
      for (int p : preds[e]) S.succ[fill[pos[p]]++] = pos[e];
    for (int k = 0; k < n; ++k)
      if (S.indeg0[k] == 0) S.ready0.push_back(k);
    preds.clear();
    preds.shrink_to_fit();
    eobjs.clear();
    eobjs.shrink_to_fit();
  }
};

}  // namespace

// ---------------------------------------------------------------- build_plan
static uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

bool build_plan(Plan& p, const double* xyz, const double* area, int64_t n64,
                const Params& prm) {
  p.prm = prm;
  int n = (int)n64;
  p.n = n;
  // cluster tree
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::vector<int64_t> order;
  order.reserve(n);
  p.cl.clear();
  p.leaves.clear();
  build_cluster(p, idx, 0, n, xyz, order);
  p.n_orig = n;
  int croot = 0;
  if (prm.operation != 0) {
    // second copy of every cluster (same boxes, offsets + n) under a new
    // root, so every quadrant of the doubled matrix has the original block
    // tree; the second copy's positions map to the same points
    const int nc = (int)p.cl.size(), nl = (int)p.leaves.size();
    for (int c = 0; c < nc; ++c) {
      Cluster c2 = p.cl[c];
      c2.off += n;
      if (c2.son[0] >= 0) {
        c2.son[0] += nc;
        c2.son[1] += nc;
      }
      if (c2.leaf >= 0) c2.leaf += nl;
      c2.first_leaf += nl;
      p.cl.push_back(c2);
    }
    for (int l = 0; l < nl; ++l) p.leaves.push_back(p.leaves[l] + nc);
    for (int i = 0; i < n; ++i) order.push_back(order[i]);
    Cluster r = p.cl[0];
    r.off = 0;
    r.size = 2 * n;
    r.son[0] = 0;
    r.son[1] = nc;
    r.leaf = -1;
    r.first_leaf = 0;
    r.nleaves = 2 * nl;
    croot = (int)p.cl.size();
    p.cl.push_back(r);
    n = 2 * n;
    p.n = n;
  }
  p.perm = order;
  p.xyz.resize((size_t)3 * n);
  p.area.resize(n);
  for (int i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) p.xyz[3 * i + d] = xyz[3 * order[i] + d];
    p.area[i] = area[order[i]];
  }
  // block tree
  p.bn.clear();
  p.blk.clear();
  p.broot = build_blocks(p, croot, croot);
  if (prm.operation != 0) {
    if (p.bn[p.broot].kind != 'H') {
      p.err = "doubled matrix without a 2 x 2 root";
      return false;
    }
    p.result_node = p.bn[p.broot].son[prm.operation == 1 ? 0 : 3];
  }

  // ---- layout of the work region: ranks | dense | low-rank
  const int es_lr = prm.mixed ? 4 : 8;
  int nR = 0, nF = 0;
  for (auto& b : p.blk) (b.kind == 'R' ? nR : nF)++;
  uint64_t cur = 0;
  p.off_status = 256;
  cur = 512;
  p.off_work = cur;
  uint64_t w = 0;
  std::vector<uint64_t> rank_rel(p.blk.size(), 0);
  for (size_t i = 0; i < p.blk.size(); ++i)
    if (p.blk[i].kind == 'R') { rank_rel[i] = w; w += 4; }
  w = align256(w);
  for (size_t i = 0; i < p.blk.size(); ++i) {
    LBlock& b = p.blk[i];
    if (b.kind == 'F') {
      b.offF = p.off_work + w;
      w = align256(w + (uint64_t)b.m * b.n * 8);
    }
  }
  for (size_t i = 0; i < p.blk.size(); ++i) {
    LBlock& b = p.blk[i];
    if (b.kind == 'R') {
      b.offRank = p.off_work + rank_rel[i];
      b.offU = p.off_work + w;
      w = align256(w + (uint64_t)b.m * prm.cap_f * es_lr);
      b.offV = p.off_work + w;
      w = align256(w + (uint64_t)b.n * prm.cap_f * es_lr);
    }
  }
  p.size_work = w;
  cur = align256(p.off_work + w);
  p.off_pristine = cur;
  cur = align256(cur + w);
  p.off_piv = cur;
  cur = align256(cur + (uint64_t)n * 4);
  p.off_inv_l = cur;
  cur = align256(cur + (uint64_t)n * 64 * 8);
  p.off_inv_u = cur;
  cur = align256(cur + (uint64_t)n * 64 * 8);

  // ---- host assembly
  Entries E{p.xyz.data(), p.area.data(), prm.kernel, p.n_orig, prm.operation, prm.kernel_b};
  p.img_work.assign(p.size_work, 0);
  std::vector<int> rids;
  for (size_t i = 0; i < p.blk.size(); ++i) rids.push_back((int)i);
  // large blocks first for load balance
  std::stable_sort(rids.begin(), rids.end(), [&](int a, int b) {
    return (int64_t)p.blk[a].m * p.blk[a].n > (int64_t)p.blk[b].m * p.blk[b].n;
  });
  std::vector<std::vector<double>> mvU(p.blk.size()), mvV(p.blk.size());
  std::atomic<int64_t> cap_hits{0};
  // cross approximation to a tenth of the tightest tolerance any copy needs
  double eps_need = prm.fixed_rank > 0 ? 1e-12 : prm.eps_f;
  if (prm.cap_mv > 0) eps_need = std::min(eps_need, prm.eps_mv);
  double eps_aca = eps_need * 0.1;
  char* img = p.img_work.data();
  if (!prm.device_asm) parallel_for((int)rids.size(), [&](int q) {
    LBlock& b = p.blk[rids[q]];
    const Cluster &ct = p.cl[b.t], &cs = p.cl[b.s];
    if (b.kind == 'F') {
      double* F = (double*)(img + (b.offF - p.off_work));
      for (int j = 0; j < b.n; ++j)
        for (int i = 0; i < b.m; ++i) F[i + (size_t)j * b.m] = E(ct.off + i, cs.off + j);
      return;
    }
    std::vector<double> U, V, Uo, Vo, sig;
    int ka = 0, r = 0;
    int kmax = std::min(std::min(b.m, b.n), 256);
    aca(E, ct.off, cs.off, b.m, b.n, eps_aca, kmax, U, V, ka);
    if (ka == 0) {
      b.kf = 0;
      b.mvk = 0;
      return;
    }
    recompress(U, V, b.m, b.n, ka, sig, Uo, Vo, r);
    bool capped;
    int kf = choose_rank(sig, prm.eps_f, prm.cap_f, prm.fixed_rank, &capped);
    if (capped) cap_hits++;
    int kmv = prm.cap_mv > 0 ? choose_rank(sig, prm.eps_mv, prm.cap_mv, 0, &capped) : 0;
    b.kf = kf;
    b.mvk = kmv;
    int32_t* rk = (int32_t*)(img + (b.offRank - p.off_work));
    *rk = kf;
    if (prm.mixed) {
      float* Ud = (float*)(img + (b.offU - p.off_work));
      float* Vd = (float*)(img + (b.offV - p.off_work));
      for (int j = 0; j < kf; ++j) {
        for (int i = 0; i < b.m; ++i) Ud[i + (size_t)j * b.m] = (float)Uo[i + (size_t)j * b.m];
        for (int i = 0; i < b.n; ++i) Vd[i + (size_t)j * b.n] = (float)Vo[i + (size_t)j * b.n];
      }
    } else {
      double* Ud = (double*)(img + (b.offU - p.off_work));
      double* Vd = (double*)(img + (b.offV - p.off_work));
      std::memcpy(Ud, Uo.data(), sizeof(double) * (size_t)b.m * kf);
      std::memcpy(Vd, Vo.data(), sizeof(double) * (size_t)b.n * kf);
    }
    mvU[rids[q]].assign(Uo.begin(), Uo.begin() + (size_t)b.m * kmv);
    mvV[rids[q]].assign(Vo.begin(), Vo.begin() + (size_t)b.n * kmv);
  });
  for (auto& b : p.blk) p.max_rank_f = std::max<int64_t>(p.max_rank_f, b.kf);

  // ---- matvec region: packed FP64 factors at their ranks
  p.off_mv = cur;
  uint64_t mw = 0;
  for (size_t i = 0; i < p.blk.size(); ++i) {
    LBlock& b = p.blk[i];
    if (b.kind != 'R') continue;
    b.mvU = p.off_mv + mw;
    mw = align256(mw + (uint64_t)b.m * b.mvk * 8);
    b.mvV = p.off_mv + mw;
    mw = align256(mw + (uint64_t)b.n * b.mvk * 8);
  }
  p.size_mv = mw;
  p.img_mv.assign(mw, 0);
  for (size_t i = 0; i < p.blk.size(); ++i) {
    LBlock& b = p.blk[i];
    if (b.kind != 'R' || b.mvk == 0) continue;
    std::memcpy(p.img_mv.data() + (b.mvU - p.off_mv), mvU[i].data(), mvU[i].size() * 8);
    std::memcpy(p.img_mv.data() + (b.mvV - p.off_mv), mvV[i].data(), mvV[i].size() * 8);
  }
  cur = align256(cur + mw);

  // ---- points in cluster order (device assembly, direct-summation residual)
  p.off_pts = cur;
  cur = align256(cur + (uint64_t)n * 4 * 8);

  // ---- device assembly: block tables, ACA workspace in chunks, and the
  // truncations that recompress each cross approximation into the factored
  // copy (C = 0 minus one term: -U_aca V_aca^T with U_aca negated)
  p.asm_dense.clear();
  p.asm_lr.clear();
  p.asm_chunks.clear();
  p.asm_ops.clear();
  p.asm_terms.clear();
  if (prm.device_asm) {
    const int KA = p.asm_kmax;
    p.asm_eps = eps_aca;
    int nlr = 0;
    for (auto& b : p.blk) nlr += b.kind == 'R';
    p.off_asm_ranks = cur;
    cur = align256(cur + (uint64_t)std::max(1, nlr) * 4);
    // workspace: at most 1 GiB (or the largest single block) per chunk
    const uint64_t cap_ws = (uint64_t)1 << 30;
    uint64_t ws = 0, ws_max = 0;
    int lr_i = 0;
    AsmChunk ch{0, 0, 0, 0};
    for (auto& b : p.blk) {
      const Cluster &ct = p.cl[b.t], &cs = p.cl[b.s];
      if (b.kind == 'F') {
        p.asm_dense.push_back(AsmBlock{b.offF, 0, 0, ct.off, cs.off, b.m, b.n});
        continue;
      }
      const uint64_t need = align256((uint64_t)b.m * KA * 8) + align256((uint64_t)b.n * KA * 8);
      if (ws > 0 && ws + need > cap_ws) {
        ch.b1 = lr_i;
        ch.op1 = (int)p.asm_ops.size();
        p.asm_chunks.push_back(ch);
        ch = AsmChunk{lr_i, lr_i, (int)p.asm_ops.size(), 0};
        ws = 0;
      }
      AsmBlock a{ws, ws + align256((uint64_t)b.m * KA * 8), p.off_asm_ranks + 4 * (uint64_t)lr_i,
                 ct.off, cs.off, b.m, b.n};   // U, V relative to the workspace for now
      ws += need;
      ws_max = std::max(ws_max, ws);
      p.asm_lr.push_back(a);
      Term t;
      std::memset(&t, 0, sizeof(t));
      t.X = PRef{a.U, a.rank, b.m, b.m, KA, DT_F64, 0, PK_MAT, 0};
      t.Y = PRef{a.V, a.rank, b.n, b.n, KA, DT_F64, 0, PK_MAT, 0};
      Op o;
      std::memset(&o, 0, sizeof(o));
      o.type = OP_TRUNC;
      o.i0 = (int32_t)p.asm_terms.size();
      o.i1 = 1;
      o.i2 = prm.cap_f | (prm.fixed_rank << 16);
      o.d0 = prm.fixed_rank > 0 ? 0.0 : prm.eps_f;
      const uint8_t dt = prm.mixed ? DT_F32 : DT_F64;
      o.p[0] = PRef{b.offU, b.offRank, b.m, b.m, prm.cap_f, dt, 0, PK_MAT, 0};
      o.p[1] = PRef{b.offV, b.offRank, b.n, b.n, prm.cap_f, dt, 0, PK_MAT, 0};
      p.asm_terms.push_back(t);
      p.asm_ops.push_back(o);
      ++lr_i;
    }
    ch.b1 = lr_i;
    ch.op1 = (int)p.asm_ops.size();
    if (ch.b1 > ch.b0) p.asm_chunks.push_back(ch);
    p.off_asm_ws = cur;
    p.size_asm_ws = align256(ws_max);
    cur = align256(cur + std::max<uint64_t>(256, p.size_asm_ws));
    for (auto& a : p.asm_lr) {
      a.U += p.off_asm_ws;
      a.V += p.off_asm_ws;
    }
    for (auto& t : p.asm_terms) {
      t.X.ptr += p.off_asm_ws;
      t.Y.ptr += p.off_asm_ws;
    }
    p.off_asm_dense = cur;
    cur = align256(cur + std::max<size_t>(1, p.asm_dense.size()) * sizeof(AsmBlock));
    p.off_asm_lr = cur;
    cur = align256(cur + std::max<size_t>(1, p.asm_lr.size()) * sizeof(AsmBlock));
    p.off_asm_ops = cur;
    cur = align256(cur + std::max<size_t>(1, p.asm_ops.size()) * sizeof(Op));
    p.off_asm_terms = cur;
    cur = align256(cur + std::max<size_t>(1, p.asm_terms.size()) * sizeof(Term));
    for (auto& o : p.asm_ops) o.p[2].ptr = p.off_asm_terms;
  }

  // ---- solve / refinement workspace
  int nr = prm.max_nrhs;
  p.off_nrhs = cur;
  cur += 256;
  p.off_Y = cur;
  cur = align256(cur + (uint64_t)n * nr * 8);
  p.off_X = cur;
  cur = align256(cur + (uint64_t)n * nr * 8);
  p.off_B = cur;
  cur = align256(cur + (uint64_t)n * nr * 8);
  p.off_eta = cur;
  cur = align256(cur + (uint64_t)4 * nr * 8 + 64);
  p.off_perm = cur;
  cur = align256(cur + (uint64_t)n * 8);
  // solve: one V^T X slot per low-rank block of the factor
  for (auto& b : p.blk)
    if (b.kind == 'R') {
      b.offT = cur;
      cur = align256(cur + (uint64_t)prm.cap_f * nr * 8);
    }
  // matvec T buffers (k_mv x nrhs per low-rank block)
  p.off_mvT = cur;
  {
    uint64_t tw = 0;
    p.mv_lr.clear();
    std::vector<uint64_t> tof(p.blk.size(), 0);
    for (size_t i = 0; i < p.blk.size(); ++i) {
      const LBlock& b = p.blk[i];
      if (b.kind != 'R') continue;
      tof[i] = p.off_mvT + tw;
      tw = align256(tw + (uint64_t)std::max(1, b.mvk) * nr * 8);
      MvLR e;
      e.U = b.mvU;
      e.V = b.mvV;
      e.T = tof[i];
      e.m = b.m;
      e.n = b.n;
      e.k = b.mvk;
      e.kcap = std::max(1, b.mvk);
      e.r0 = p.cl[b.t].off;
      e.c0 = p.cl[b.s].off;
      p.mv_lr.push_back(e);
    }
    cur = align256(cur + tw);
    // per leaf row lists
    std::vector<std::vector<MvTerm>> rows(p.leaves.size());
    for (size_t i = 0; i < p.blk.size(); ++i) {
      const LBlock& b = p.blk[i];
      const Cluster& ct = p.cl[b.t];
      for (int l = ct.first_leaf; l < ct.first_leaf + ct.nleaves; ++l) {
        const Cluster& lc = p.cl[p.leaves[l]];
        MvTerm t;
        t.roff = lc.off - ct.off;
        if (b.kind == 'F') {
          // the working copy is overwritten by the factorisation: the
          // matvec reads the near field from the pristine copy
          t.A = b.offF - p.off_work + p.off_pristine;
          t.T = 0;
          t.lda = b.m;
          t.ncol = b.n;
          t.c0 = p.cl[b.s].off;
        } else {
          if (b.mvk == 0) continue;
          t.A = b.mvU;
          t.T = tof[i];
          t.lda = b.m;
          t.ncol = b.mvk;
          t.c0 = std::max(1, b.mvk);
        }
        rows[l].push_back(t);
      }
    }
    p.mv_terms.clear();
    p.mv_rows.clear();
    for (size_t l = 0; l < p.leaves.size(); ++l) {
      const Cluster& lc = p.cl[p.leaves[l]];
      MvRow r{lc.off, lc.size, (int32_t)p.mv_terms.size(), (int32_t)rows[l].size()};
      p.mv_rows.push_back(r);
      for (auto& t : rows[l]) p.mv_terms.push_back(t);
    }
  }

  // ---- schedules
  p.off_scratch = cur;
  {
    Builder B(p, p.fsched);
    B.P_dt = prm.mixed ? DT_F32 : DT_F64;
    B.chunk_cols = std::max(1, 64 - prm.cap_f);
    B.scratch_base = p.off_scratch;
    B.ring_cap = prm.scratch_cap & ~(uint64_t)255;
    for (auto& b : p.blk) {
      int rows_cl = b.t;
      if (b.kind == 'F') b.objF = B.new_obj(-1, true);
      else {
        b.objU = B.new_obj(rows_cl, false);
        b.objV = B.new_obj(b.s, false);
        b.objRank = B.new_obj(-1, true);
      }
    }
    B.cost_cur = 0;
    if (prm.operation == 0) {
      B.lu(p.broot);
    } else {
      const BNode& R = p.bn[p.broot];
      const int q00 = R.son[0], q01 = R.son[1], q10 = R.son[2], q11 = R.son[3];
      if (prm.operation == 1) {
        B.gemm(q00, q01, q10);
      } else {
        B.lu(q00);
        B.trsm_l(q00, q01);
        B.trsm_u(q10, q00);
        B.gemm(q11, q10, q01);
      }
    }
    if (!p.err.empty()) return false;
    B.finish();
    if (std::getenv("HLU_DEBUG"))
      std::fprintf(stderr, "[hlu] gemm calls %lld, truncation groups (call, target) %zu\n",
                   (long long)B.call_id, B.trunc_groups.size());
    p.size_scratch = align256(B.scratch_cur);
    cur = align256(p.off_scratch + p.size_scratch);
    p.off_cost = cur;
    // patch op cost records to absolute offsets
    for (auto& op : p.fsched.ops) op.cost += p.off_cost;
    cur = align256(cur + (uint64_t)p.fsched.ops.size() * kCostRecBytes);
  }
  {
    Builder B(p, p.ssched);
    B.P_dt = prm.mixed ? DT_F32 : DT_F64;
    B.solve_mv = true;
    B.cost_cur = 0;
    for (auto& b : p.blk) {
      if (b.kind == 'F') b.objF = B.new_obj(-1, true);
      else {
        b.objU = B.new_obj(b.t, false);
        b.objV = B.new_obj(b.s, false);
        b.objRank = B.new_obj(-1, true);
      }
    }
    PV Y;
    Y.obj = B.new_obj(0, false);
    Y.off = p.off_Y;
    Y.ld = n;
    Y.rows = n;
    Y.cols = nr;
    Y.rank = p.off_nrhs;
    Y.cl = 0;
    Y.dt = DT_F64;
    if (prm.operation == 0) {
      B.fwd(p.broot, Y);
      B.bwd(p.broot, Y);
    }
    B.finish();
    p.off_cost_s = cur;
    for (auto& op : p.ssched.ops) op.cost += p.off_cost_s;
    cur = align256(cur + (uint64_t)p.ssched.ops.size() * kCostRecBytes);
  }
  p.off_ops_f = cur;
  cur = align256(cur + p.fsched.ops.size() * sizeof(Op));
  p.off_ops_s = cur;
  cur = align256(cur + p.ssched.ops.size() * sizeof(Op));
  p.off_terms_f = cur;
  cur = align256(cur + std::max<size_t>(1, p.fsched.terms.size()) * sizeof(Term));
  for (auto& op : p.fsched.ops)
    if (op.type == OP_TRUNC) op.p[2].ptr = p.off_terms_f;
  p.off_terms_s = cur;
  cur = align256(cur + std::max<size_t>(1, p.ssched.terms.size()) * sizeof(Term));
  for (auto& op : p.ssched.ops)
    if (op.type == OP_MVROW) {
      if (op.i1 == 1) {
        // one term: carried in the op (p1 its factor, p2 its operand, i0 = -1),
        // so its loads need not wait for a term record
        const Term& tm = p.ssched.terms[op.i0];
        op.p[1] = tm.X;
        op.p[2] = tm.Y;
        op.i0 = -1;
      } else {
        op.p[2].ptr = p.off_terms_s;
      }
    }
  {
    const uint64_t N = p.fsched.ops.size();
    p.off_df_succ_off = cur;
    cur = align256(cur + (N + 1) * 4);
    p.off_df_succ = cur;
    cur = align256(cur + std::max<uint64_t>(1, p.fsched.succ.size()) * 4);
    p.off_df_indeg0 = cur;
    cur = align256(cur + std::max<uint64_t>(1, N) * 4);
    p.off_df_indeg = cur;
    cur = align256(cur + std::max<uint64_t>(1, N) * 4);
    p.off_df_queue = cur;
    cur = align256(cur + std::max<uint64_t>(1, N) * 4);
    p.off_df_ready0 = cur;
    cur = align256(cur + std::max<uint64_t>(1, p.fsched.ready0.size()) * 4);
    p.off_df_ctrl = cur;
    cur = align256(cur + 256);
  }
  {
    const uint64_t N = p.ssched.ops.size();
    p.off_dfs_succ_off = cur;
    cur = align256(cur + (N + 1) * 4);
    p.off_dfs_succ = cur;
    cur = align256(cur + std::max<uint64_t>(1, p.ssched.succ.size()) * 4);
    p.off_dfs_indeg0 = cur;
    cur = align256(cur + std::max<uint64_t>(1, N) * 4);
    p.off_dfs_indeg = cur;
    cur = align256(cur + std::max<uint64_t>(1, N) * 4);
    p.off_dfs_queue = cur;
    cur = align256(cur + std::max<uint64_t>(1, N) * 4);
    p.off_dfs_ready0 = cur;
    cur = align256(cur + std::max<uint64_t>(1, p.ssched.ready0.size()) * 4);
    p.off_dfs_ctrl = cur;
    cur = align256(cur + 256);
  }
  p.off_mv_lr = cur;
  cur = align256(cur + p.mv_lr.size() * sizeof(MvLR));
  p.off_mv_terms = cur;
  cur = align256(cur + p.mv_terms.size() * sizeof(MvTerm));
  p.off_mv_rows = cur;
  cur = align256(cur + p.mv_rows.size() * sizeof(MvRow));
  p.total = cur;
  (void)cap_hits;
  (void)nF;
  (void)nR;
  return true;
}

}  // namespace hlu
