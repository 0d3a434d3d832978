// Host FP64 precomputation for the bbFMM M2L. See host_math.h.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace bbfmm {

std::vector<double> cheb_nodes(int order) {
  std::vector<double> x(order);
  for (int k = 1; k <= order; ++k) x[k - 1] = -std::cos((2.0 * k - 1.0) * M_PI / (2.0 * order));
  return x;
}

double cheb_basis(int order, double u, int m) {
  // T_k by the three-term recurrence at u and at the node.
  const double xm = -std::cos((2.0 * (m + 1) - 1.0) * M_PI / (2.0 * order));
  double tu0 = 1.0, tu1 = u, tx0 = 1.0, tx1 = xm;
  double sum = 1.0 / order;
  for (int k = 1; k < order; ++k) {
    sum += (2.0 / order) * tu1 * tx1;
    const double tu2 = 2.0 * u * tu1 - tu0, tx2 = 2.0 * xm * tx1 - tx0;
    tu0 = tu1; tu1 = tu2; tx0 = tx1; tx1 = tx2;
  }
  return sum;
}

double kernel_value(int kind, double c, double r) {
  switch (kind) {
    case kInvR: return r > 0.0 ? 1.0 / r : 0.0;
    case kInvSqrtR2C2: return 1.0 / std::sqrt(r * r + c * c);
    case kHelmCos: return r > 0.0 ? std::cos(c * r) / r : 0.0;
    case kHelmSin: return r > 0.0 ? std::sin(c * r) / r : c;
    case kR2: return r * r;
    case kR4: return (r * r) * (r * r);
    default: return 0.0;
  }
}

bool kernel_is_homogeneous(int kind, double* degree) {
  switch (kind) {
    case kInvR: *degree = -1.0; return true;
    case kR2: *degree = 2.0; return true;
    case kR4: *degree = 4.0; return true;
    default: *degree = 0.0; return false;
  }
}

const std::array<std::array<int, 3>, kNumSym>& representatives() {
  static const std::array<std::array<int, 3>, kNumSym> reps = [] {
    std::array<std::array<int, 3>, kNumSym> r{};
    int n = 0;
    for (int a = 2; a <= 3; ++a)
      for (int b = 0; b <= a; ++b)
        for (int c = 0; c <= b; ++c) r[n++] = {a, b, c};
    return r;
  }();
  return reps;
}

const std::array<std::array<int, 3>, 6>& axis_orders() {
  static const std::array<std::array<int, 3>, 6> ord = {{{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                                          {1, 2, 0}, {2, 0, 1}, {2, 1, 0}}};
  return ord;
}

SymInfo symmetry_of(const int t[3]) {
  SymInfo s{};
  int at[3];
  for (int r = 0; r < 3; ++r) {
    if (t[r] < 0) s.flip |= 1 << r;
    at[r] = std::abs(t[r]);
  }
  // Stable descending order of |t|: insertion sort on axis indices.
  int ax[3] = {0, 1, 2};
  for (int i = 1; i < 3; ++i)
    for (int j = i; j > 0 && at[ax[j]] > at[ax[j - 1]]; --j) std::swap(ax[j], ax[j - 1]);
  const auto& ords = axis_orders();
  for (int k = 0; k < 6; ++k)
    if (ords[k][0] == ax[0] && ords[k][1] == ax[1] && ords[k][2] == ax[2]) s.axes = k;
  const int pt[3] = {at[ax[0]], at[ax[1]], at[ax[2]]};
  const auto& reps = representatives();
  s.p = -1;
  for (int k = 0; k < kNumSym; ++k)
    if (reps[k][0] == pt[0] && reps[k][1] == pt[1] && reps[k][2] == pt[2]) s.p = k;
  s.perm_id = s.flip * 6 + s.axes;
  return s;
}

void sigma_table(int order, int perm_id, int32_t* out) {
  const int flip = perm_id / 6;
  const auto& ax = axis_orders()[perm_id % 6];
  const int nn = order * order * order;
  for (int i = 0; i < nn; ++i) {
    int a[3] = {i % order, (i / order) % order, i / (order * order)};
    for (int r = 0; r < 3; ++r)
      if (flip & (1 << r)) a[r] = order - 1 - a[r];
    out[i] = a[ax[0]] + order * a[ax[1]] + order * order * a[ax[2]];
  }
}

void m2l_operator(int kind, double c, int order, double width, int p, double* out) {
  const std::vector<double> x = cheb_nodes(order);
  const auto& t = representatives()[p];
  const int nn = order * order * order;
  for (int i = 0; i < nn; ++i) {
    const int a[3] = {i % order, (i / order) % order, i / (order * order)};
    for (int j = 0; j < nn; ++j) {
      const int b[3] = {j % order, (j / order) % order, j / (order * order)};
      double r2 = 0.0;
      for (int s = 0; s < 3; ++s) {
        const double d = width * t[s] + 0.5 * width * (x[a[s]] - x[b[s]]);
        r2 += d * d;
      }
      out[(size_t)i * nn + j] = kernel_value(kind, c, std::sqrt(r2));
    }
  }
}

void jacobi_svd(const double* a, int m, int n, double* u, double* s, double* v) {
  // Work column-major: column j of A in w[j*m .. j*m+m).
  std::vector<double> w((size_t)m * n), vv((size_t)n * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) w[(size_t)j * m + i] = a[(size_t)i * n + j];
  for (int j = 0; j < n; ++j) vv[(size_t)j * n + j] = 1.0;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      double* wp = &w[(size_t)p * m];
      for (int q = p + 1; q < n; ++q) {
        double* wq = &w[(size_t)q * m];
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int k = 0; k < m; ++k) {
          alpha += wp[k] * wp[k];
          beta += wq[k] * wq[k];
          gamma += wp[k] * wq[k];
        }
        if (gamma == 0.0 || std::fabs(gamma) <= tol * std::sqrt(alpha * beta)) continue;
        rotated = true;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int k = 0; k < m; ++k) {
          const double x0 = wp[k], x1 = wq[k];
          wp[k] = cs * x0 - sn * x1;
          wq[k] = sn * x0 + cs * x1;
        }
        double* vp = &vv[(size_t)p * n];
        double* vq = &vv[(size_t)q * n];
        for (int k = 0; k < n; ++k) {
          const double x0 = vp[k], x1 = vq[k];
          vp[k] = cs * x0 - sn * x1;
          vq[k] = sn * x0 + cs * x1;
        }
      }
    }
    if (!rotated) break;
  }
  std::vector<double> norms(n);
  for (int j = 0; j < n; ++j) {
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += w[(size_t)j * m + k] * w[(size_t)j * m + k];
    norms[j] = std::sqrt(acc);
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return norms[x] > norms[y]; });
  for (int jj = 0; jj < n; ++jj) {
    const int j = idx[jj];
    s[jj] = norms[j];
    const double inv = norms[j] > 0.0 ? 1.0 / norms[j] : 0.0;
    for (int k = 0; k < m; ++k) u[(size_t)k * n + jj] = w[(size_t)j * m + k] * inv;
    for (int k = 0; k < n; ++k) v[(size_t)k * n + jj] = vv[(size_t)j * n + k];
  }
}

int truncation_rank(const double* s, int n, double eps) {
  if (n == 0 || s[0] == 0.0) return 0;
  int r = 0;
  for (int k = 0; k < n; ++k)
    if (s[k] > eps * s[0]) ++r;
  if (r < 1) r = 1;
  while (r < n && std::fabs(s[r] - s[r - 1]) <= 1e-10 * s[0]) ++r;
  return r;
}

void householder_qr(const double* a, long long m, int n, double* q, double* r) {
  // Column-major work copy; reflectors kept in the lower part, their scalars in beta.
  std::vector<double> w((size_t)m * n), beta(n, 0.0), diag(n, 0.0);
  for (long long i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) w[(size_t)j * m + i] = a[(size_t)i * n + j];
  for (int j = 0; j < n; ++j) {
    double* col = &w[(size_t)j * m];
    double norm2 = 0.0;
    for (long long i = j; i < m; ++i) norm2 += col[i] * col[i];
    const double norm = std::sqrt(norm2);
    if (norm == 0.0) {
      diag[j] = 0.0;
      continue;
    }
    const double alpha = col[j] >= 0.0 ? -norm : norm;
    // v = x - alpha e_1 stored in col[j..m), H = I - beta v v^T
    col[j] -= alpha;
    const double vnorm2 = norm2 - 2.0 * alpha * (col[j] + alpha) + alpha * alpha;
    beta[j] = vnorm2 > 0.0 ? 2.0 / vnorm2 : 0.0;
    diag[j] = alpha;
    for (int c = j + 1; c < n; ++c) {
      double* cc = &w[(size_t)c * m];
      double dot = 0.0;
      for (long long i = j; i < m; ++i) dot += col[i] * cc[i];
      dot *= beta[j];
      for (long long i = j; i < m; ++i) cc[i] -= dot * col[i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) r[(size_t)i * n + j] = j < i ? 0.0 : (j == i ? diag[i] : w[(size_t)j * m + i]);
  if (!q) return;
  // Q = H_0 H_1 ... H_{n-1} applied to the first n columns of the identity
  std::vector<double> qc((size_t)m * n, 0.0);
  for (int j = 0; j < n; ++j) qc[(size_t)j * m + j] = 1.0;
  for (int h = n - 1; h >= 0; --h) {
    if (beta[h] == 0.0) continue;
    const double* v = &w[(size_t)h * m];
    for (int c = 0; c < n; ++c) {
      double* cc = &qc[(size_t)c * m];
      double dot = 0.0;
      for (long long i = h; i < m; ++i) dot += v[i] * cc[i];
      dot *= beta[h];
      for (long long i = h; i < m; ++i) cc[i] -= dot * v[i];
    }
  }
  for (long long i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) q[(size_t)i * n + j] = qc[(size_t)j * m + i];
}

namespace {

// First index among `allowed` whose |x| lies within min(window, m / 2) of the largest, m; -1 if
// none. Mirror-image kernel entries are equal in exact arithmetic and a residual's rounding error
// scales with the matrix's largest entry, so ties are judged on that scale (window).
int tied_argmax(const double* x, int n, const std::vector<char>* allowed, double window, double* max_out) {
  double m = -1.0;
  for (int i = 0; i < n; ++i)
    if (!allowed || (*allowed)[i]) m = std::max(m, std::fabs(x[i]));
  *max_out = m;
  if (m < 0.0) return -1;
  const double cut = m - std::min(window, 0.5 * m);
  for (int i = 0; i < n; ++i)
    if ((!allowed || (*allowed)[i]) && std::fabs(x[i]) >= cut) return i;
  return -1;
}

double dot(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

}  // namespace

int aca_partial(const double* k, int n, double tol, std::vector<double>& u, std::vector<double>& v) {
  u.clear();
  v.clear();
  std::vector<char> free_row(n, 1);
  std::vector<double> row(n), col(n);
  int nfree = n, i = 0, crosses = 0;
  double norm2 = 0.0, kmax = 0.0;
  for (size_t e = 0; e < (size_t)n * n; ++e) kmax = std::max(kmax, std::fabs(k[e]));
  const double window = 1e-12 * kmax;
  while (crosses < n) {
    if (free_row[i]) {
      free_row[i] = 0;
      --nfree;
    }
    for (int j = 0; j < n; ++j) row[j] = k[(size_t)i * n + j];
    for (int l = 0; l < crosses; ++l) {
      const double ui = u[(size_t)l * n + i];
      const double* vl = &v[(size_t)l * n];
      for (int j = 0; j < n; ++j) row[j] -= ui * vl[j];
    }
    double rmax;
    const int jp = tied_argmax(row.data(), n, nullptr, window, &rmax);
    if (rmax == 0.0) {
      if (nfree == 0) break;
      i = (int)(std::find(free_row.begin(), free_row.end(), 1) - free_row.begin());
      continue;
    }
    const double piv = row[jp];
    for (int j = 0; j < n; ++j) row[j] /= piv;
    for (int r = 0; r < n; ++r) col[r] = k[(size_t)r * n + jp];
    for (int l = 0; l < crosses; ++l) {
      const double vj = v[(size_t)l * n + jp];
      const double* ul = &u[(size_t)l * n];
      for (int r = 0; r < n; ++r) col[r] -= vj * ul[r];
    }
    const double uu = dot(col.data(), col.data(), n), vv = dot(row.data(), row.data(), n);
    for (int l = 0; l < crosses; ++l)
      norm2 += 2.0 * dot(col.data(), &u[(size_t)l * n], n) * dot(row.data(), &v[(size_t)l * n], n);
    norm2 += uu * vv;
    u.insert(u.end(), col.begin(), col.end());
    v.insert(v.end(), row.begin(), row.end());
    ++crosses;
    if (std::sqrt(uu * vv) <= tol * std::sqrt(norm2) || nfree == 0) break;
    double umax;
    i = tied_argmax(col.data(), n, &free_row, window, &umax);
  }
  return crosses;
}

int compress_svd(const double* k, int n, double eps, std::vector<double>& uf, std::vector<double>& vf) {
  std::vector<double> U((size_t)n * n), S(n), V((size_t)n * n);
  jacobi_svd(k, n, n, U.data(), S.data(), V.data());
  const int r = truncation_rank(S.data(), n, eps);
  uf.assign((size_t)n * r, 0.0);
  vf.assign((size_t)n * r, 0.0);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < r; ++c) {
      uf[(size_t)i * r + c] = U[(size_t)i * n + c] * S[c];
      vf[(size_t)i * r + c] = V[(size_t)i * n + c];
    }
  return r;
}

int compress_aca(const double* k, int n, const int32_t* q, double eps, std::vector<double>& uf,
                 std::vector<double>& vf) {
  std::vector<double> cu, cv;
  const int nc = aca_partial(k, n, kAcaRelTol * eps, cu, cv);
  // A_s = 1/2 [U, V_Q] [V, U_Q]^T with U_Q[i] = U[Q(i)] (row-major n x 2nc factors)
  const int m2 = 2 * nc;
  if (m2 == 0) {
    uf.clear();
    vf.clear();
    return 0;
  }
  std::vector<double> fa((size_t)n * m2), fb((size_t)n * m2);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < nc; ++l) {
      fa[(size_t)i * m2 + l] = cu[(size_t)l * n + i];
      fa[(size_t)i * m2 + nc + l] = cv[(size_t)l * n + q[i]];
      fb[(size_t)i * m2 + l] = 0.5 * cv[(size_t)l * n + i];
      fb[(size_t)i * m2 + nc + l] = 0.5 * cu[(size_t)l * n + q[i]];
    }
  if (m2 >= n) {
    // as many factor columns as rows: truncate the dense sum directly
    std::vector<double> a((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) a[(size_t)i * n + j] = dot(&fa[(size_t)i * m2], &fb[(size_t)j * m2], m2);
    return compress_svd(a.data(), n, eps, uf, vf);
  }
  std::vector<double> qa((size_t)n * m2), ra((size_t)m2 * m2), qb((size_t)n * m2), rb((size_t)m2 * m2);
  householder_qr(fa.data(), n, m2, qa.data(), ra.data());
  householder_qr(fb.data(), n, m2, qb.data(), rb.data());
  // core C = Ra Rb^T, C = X Sigma Y^T, A_s = (Qa X) Sigma (Qb Y)^T
  std::vector<double> core((size_t)m2 * m2);
  for (int i = 0; i < m2; ++i)
    for (int j = 0; j < m2; ++j) core[(size_t)i * m2 + j] = dot(&ra[(size_t)i * m2], &rb[(size_t)j * m2], m2);
  std::vector<double> X((size_t)m2 * m2), S(m2), Y((size_t)m2 * m2);
  jacobi_svd(core.data(), m2, m2, X.data(), S.data(), Y.data());
  const int r = truncation_rank(S.data(), m2, eps);
  uf.assign((size_t)n * r, 0.0);
  vf.assign((size_t)n * r, 0.0);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < r; ++c) {
      double a = 0.0, b = 0.0;
      for (int l = 0; l < m2; ++l) {
        a += qa[(size_t)i * m2 + l] * X[(size_t)l * m2 + c];
        b += qb[(size_t)i * m2 + l] * Y[(size_t)l * m2 + c];
      }
      uf[(size_t)i * r + c] = a * S[c];
      vf[(size_t)i * r + c] = b;
    }
  return r;
}

void sa_operators(int kind, double c, int order, double width, double eps, bool recompress, SAOperators& out) {
  const int n = order * order * order;
  out = SAOperators();
  out.n = n;
  std::vector<std::vector<double>> kp(kNumSym, std::vector<double>((size_t)n * n));
  for (int p = 0; p < kNumSym; ++p) m2l_operator(kind, c, order, width, p, kp[p].data());
  // the 316 codes and their operators K_t[i][j] = K_p[sigma(i)][sigma(j)], t = -d
  std::vector<int> codes;
  for (int code = 0; code < 512; ++code) {
    const int f[3] = {code & 7, (code >> 3) & 7, (code >> 6) & 7};
    if (f[0] > 6 || f[1] > 6 || f[2] > 6) continue;
    if (std::max({std::abs(f[0] - 3), std::abs(f[1] - 3), std::abs(f[2] - 3)}) < 2) continue;
    codes.push_back(code);
  }
  auto operator_of = [&](int code, std::vector<double>& kt, std::vector<int32_t>& sg) {
    const int t[3] = {3 - (code & 7), 3 - ((code >> 3) & 7), 3 - ((code >> 6) & 7)};
    const SymInfo si = symmetry_of(t);
    sigma_table(order, si.perm_id, sg.data());
    const std::vector<double>& k = kp[si.p];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) kt[(size_t)i * n + j] = k[(size_t)sg[i] * n + sg[j]];
  };
  // stacked K_t^T: (316 n) x n, row-major
  const long long m = (long long)codes.size() * n;
  std::vector<double> stack((size_t)m * n), kt((size_t)n * n);
  std::vector<int32_t> sg(n);
  for (size_t b = 0; b < codes.size(); ++b) {
    operator_of(codes[b], kt, sg);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) stack[((size_t)b * n + j) * n + i] = kt[(size_t)i * n + j];
  }
  std::vector<double> R((size_t)n * n);
  householder_qr(stack.data(), m, n, nullptr, R.data());
  std::vector<double>().swap(stack);
  // K^(row) K^(row)^T = R^T R: U = the right singular vectors of R
  std::vector<double> ur((size_t)n * n), vr((size_t)n * n);
  out.sigma.assign(n, 0.0);
  jacobi_svd(R.data(), n, n, ur.data(), out.sigma.data(), vr.data());
  const int r = truncation_rank(out.sigma.data(), n, eps);
  out.r = r;
  out.u.assign((size_t)n * r, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < r; ++k) out.u[(size_t)i * r + k] = vr[(size_t)i * n + k];
  out.core.assign(512, {});
  out.ubar.assign(512, {});
  out.vbar.assign(512, {});
  std::vector<double> ku((size_t)n * r), C((size_t)r * r);
  std::vector<double> X((size_t)r * r), S(r), Y((size_t)r * r);
  for (int code : codes) {
    operator_of(code, kt, sg);
    // C_t = U^T (K_t U), loops ordered for unit-stride inner products
    std::fill(ku.begin(), ku.end(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double kij = kt[(size_t)i * n + j];
        const double* uj = &out.u[(size_t)j * r];
        double* ki = &ku[(size_t)i * r];
        for (int k = 0; k < r; ++k) ki[k] += kij * uj[k];
      }
    std::fill(C.begin(), C.end(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < r; ++a) {
        const double uia = out.u[(size_t)i * r + a];
        const double* ki = &ku[(size_t)i * r];
        double* ca = &C[(size_t)a * r];
        for (int b = 0; b < r; ++b) ca[b] += uia * ki[b];
      }
    out.rank[code] = r;
    if (recompress) {
      jacobi_svd(C.data(), r, r, X.data(), S.data(), Y.data());
      const int rt = truncation_rank(S.data(), r, eps);
      if (2 * rt < r) {
        out.rank[code] = rt;
        std::vector<double>& ub = out.ubar[code];
        std::vector<double>& vb = out.vbar[code];
        ub.assign((size_t)r * rt, 0.0);
        vb.assign((size_t)r * rt, 0.0);
        for (int a = 0; a < r; ++a)
          for (int q = 0; q < rt; ++q) {
            ub[(size_t)a * rt + q] = X[(size_t)a * r + q] * S[q];
            vb[(size_t)a * rt + q] = Y[(size_t)a * r + q];
          }
        continue;
      }
    }
    out.core[code] = C;
  }
}

void octant_table(int octant, int32_t* entries, int32_t* group_start) {
  const int o[3] = {octant & 1, (octant >> 1) & 1, (octant >> 2) & 1};
  struct E { int d[3]; int p; int perm; int order; };
  std::vector<E> list;
  int seq = 0;
  for (int dz = -3; dz <= 3; ++dz)
    for (int dy = -3; dy <= 3; ++dy)
      for (int dx = -3; dx <= 3; ++dx) {
        const int d[3] = {dx, dy, dz};
        bool ok = true;
        int linf = 0;
        for (int r = 0; r < 3; ++r) {
          // target coordinate 2P + o, source 2P + o + d; parents must be neighbours.
          const int num = o[r] + d[r];
          const int pshift = (num >= 0) ? num / 2 : -((-num + 1) / 2);  // floor(num / 2)
          if (pshift < -1 || pshift > 1) ok = false;
          linf = std::max(linf, std::abs(d[r]));
        }
        if (!ok || linf <= 1) continue;
        const int t[3] = {-dx, -dy, -dz};
        const SymInfo si = symmetry_of(t);
        list.push_back(E{{dx, dy, dz}, si.p, si.perm_id, seq++});
      }
  std::stable_sort(list.begin(), list.end(), [](const E& a, const E& b) { return a.p < b.p; });
  for (int p = 0; p <= kNumSym; ++p) group_start[p] = 0;
  for (size_t k = 0; k < list.size() && k < (size_t)kFarPerOctant; ++k) {
    const E& e = list[k];
    entries[k] = (e.d[0] + 3) | ((e.d[1] + 3) << 3) | ((e.d[2] + 3) << 6) | (e.p << 9) |
                 (e.perm << 13);
  }
  int cursor = 0;
  for (int p = 0; p < kNumSym; ++p) {
    group_start[p] = cursor;
    for (const E& e : list)
      if (e.p == p) ++cursor;
  }
  group_start[kNumSym] = cursor;
}

}  // namespace bbfmm
