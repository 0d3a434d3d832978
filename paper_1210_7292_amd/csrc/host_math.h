// Host-side FP64 precomputation of the bbFMM (pure C++, no HIP): Chebyshev interpolation,
// M2L operators of the 16 representative transfer vectors, their truncated SVD, and the
// symmetry tables that map every transfer vector onto a representative.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

namespace bbfmm {

constexpr int kMaxOrder = 9;
constexpr int kNumSym = 16;      // |T_sym| (Eq. reduced_interaction_list)
constexpr int kNumPerms = 48;    // 8 axial reflections x 6 axis orders
constexpr int kFarPerOctant = 189;

enum KernelKind : int32_t { kInvR = 0, kInvSqrtR2C2 = 1, kHelmCos = 2, kHelmSin = 3, kR2 = 100, kR4 = 101 };

// Chebyshev roots of T_l, ascending (Sec. 2.1; T_l(x) = cos(l arccos x)).
std::vector<double> cheb_nodes(int order);

// S_l(u, xbar_m) in the Chebyshev-sum form 1/l + 2/l sum_{k=1}^{l-1} T_k(u) T_k(xbar_m).
double cheb_basis(int order, double u, int m);

// Kernel value at distance r (c: the regularisation of kInvSqrtR2C2, the wavenumber of the
// Helmholtz parts).
double kernel_value(int kind, double c, double r);
bool kernel_is_homogeneous(int kind, double* degree);

// The 16 representatives t1 >= t2 >= t3 >= 0 with max(t) in {2, 3}, in a fixed order.
const std::array<std::array<int, 3>, kNumSym>& representatives();

// The 6 axis orders (lexicographic permutations of {0, 1, 2}).
const std::array<std::array<int, 3>, 6>& axis_orders();

struct SymInfo {
  int p;        // index into representatives()
  int flip;     // bit r set when t_r < 0 (Eq. axial_permutation)
  int axes;     // index into axis_orders(): |t_{a0}| >= |t_{a1}| >= |t_{a2}|, ties by axis
  int perm_id;  // flip * 6 + axes, 0..47
};
SymInfo symmetry_of(const int t[3]);

// sigma for permutation id `perm_id`: K_t[i][j] = K_p[sigma[i]][sigma[j]].
// sigma(i) = m(pi(flip(m^{-1}(i)))), pi(a)_s = a_{axes[s]}, m(a) = a0 + l a1 + l^2 a2.
void sigma_table(int order, int perm_id, int32_t* out);

// Full M2L operator of representative p at cell width `width` (row-major l^3 x l^3):
// K[m(a)][n(b)] = K(width * t_p + width/2 * (xhat_a - xhat_b)).
void m2l_operator(int kind, double c, int order, double width, int p, double* out);

// One-sided (Hestenes) Jacobi SVD of a row-major m x n matrix (m >= n):
// A = U diag(S) V^T, U m x n (row-major), S descending, V n x n (row-major).
void jacobi_svd(const double* a, int m, int n, double* u, double* s, double* v);

// Rank rule: count of s_k > eps * s_0, extended over values within 1e-10 * s_0 of the last kept.
int truncation_rank(const double* s, int n, double eps);

// Householder QR of a row-major m x n matrix (m >= n): A = Q R with Q m x n (orthonormal
// columns) and R n x n upper triangular, both row-major. Rank-deficient input is fine. q may be
// null (R only).
void householder_qr(const double* a, long long m, int n, double* q, double* r);

// Adaptive cross approximation with partial pivoting of a row-major n x n matrix (Sec. 4.1 and
// Sec. 5 name ACA as the faster replacement of the SVD): crosses u_k, v_k (each n doubles,
// appended to u and v) with K ~ sum_k u_k v_k^T. Pivot row first 0, then the largest |u_k(i)|
// over unused rows; pivot column the largest entry of the residual row; candidates within
// 1e-12 max|K| (at most half the largest) of the largest count as tied and the first index wins.
// Stops when
// ||u_k|| ||v_k|| <= tol ||S_k||_F (S_k the sum so far) or when every row has been used; a
// residual row that is exactly zero is skipped. Returns the number of crosses.
int aca_partial(const double* k, int n, double tol, std::vector<double>& u, std::vector<double>& v);

// Compressed operator K ~ Uf Vf^T (row-major n x r each, Uf = U_r Sigma_r, Vf = V_r); returns r.
// Truncated SVD of K (Eq. ialowrank):
int compress_svd(const double* k, int n, double eps, std::vector<double>& uf, std::vector<double>& vf);
// ACA (tolerance 1e-2 eps) followed by a truncated SVD at eps. The ACA sum A is first made
// consistent with the exact operator's K^T = K[Q][:, Q] (q: the involution Q, n entries) as
// (A[i][j] + A[Q(j)][Q(i)]) / 2, so that the compressed operators of t and -t stay transposes;
// the SVD of that rank-2k sum is taken from the QR factors of its two factor matrices.
int compress_aca(const double* k, int n, const int32_t* q, double eps, std::vector<double>& uf,
                 std::vector<double>& vf);
constexpr double kAcaRelTol = 1e-2;

// Single low-rank approximation (SA) of the 316 far-field operators of one cell width and its
// recompressed form (SArcmp), Sec. 4.1: U = the left singular vectors of K^(row) = [K_1, ...,
// K_316] truncated by `truncation_rank` at eps (rank r); for the symmetric kernels here the
// right singular vectors B of K^(col) span the same space, so B = U and each operator is
// K_t ~ U C_t U^T with C_t = U^T K_t U (Eq. ucb_no_compression). With recompression, C_t is
// replaced by its truncated SVD Ubar_t Vbar_t^T (rank r_t by `truncation_rank` relative to C_t's
// largest singular value) when r_t < r/2 (Eq. recompression). U is taken from a Householder QR
// of the stacked K_t^T (316 l^3 x l^3) and a Jacobi SVD of its R factor.
// Operators are indexed by the offset code of d = Y - X = -t: (dx+3) | (dy+3) << 3 | (dz+3) << 6.
struct SAOperators {
  int n = 0, r = 0;
  std::vector<double> u;                     // n x r, row-major
  std::vector<double> sigma;                 // singular values of K^(row), descending (n)
  std::array<int, 512> rank{};               // 0: not a far-field code; r: C_t kept; else r_t
  std::vector<std::vector<double>> core;     // per code, rank == r: C_t (r x r, row-major)
  std::vector<std::vector<double>> ubar, vbar;  // per code, rank < r: r x r_t each, row-major
};
void sa_operators(int kind, double c, int order, double width, double eps, bool recompress, SAOperators& out);

// Far-field table of a target octant (x bit 0, y bit 1, z bit 2): the 189 source offsets
// d = Y - X (cell units) whose source is a child of a neighbour of the target's parent and not a
// neighbour of the target, sorted by representative (stable). Each entry packs
// (dx+3) | (dy+3) << 3 | (dz+3) << 6 | p << 9 | perm_id << 13, where t = -d.
// group_start[p] .. group_start[p+1] delimits representative p.
void octant_table(int octant, int32_t* entries /*189*/, int32_t* group_start /*17*/);

}  // namespace bbfmm
