// Host FP64 dense kernels for the small matrices of LOBPCG: the Cholesky
// factorisations of steps 3, 11 and 14 and the Rayleigh-Ritz eigenproblem of
// step 24 (Section 2.2).  The matrices are at most 3m x 3m, so they stay on the
// host in FP64, as the paper's implementation does with LAPACK.
//
// Symmetric eigensolver: Householder reduction to tridiagonal form followed by
// the implicit symmetric QR iteration with Wilkinson shift (Golub & Van Loan,
// Matrix Computations, Algorithms 8.3.1 and 8.3.3), written for this library.
#include "dense.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace lobpcg {

// Scale-invariant Cholesky: with D = diag(G)^(1/2), factor Gh = D^-1 G D^-1 =
// Rh^T Rh and return R = Rh D.  Section 2.2 stresses that the factorisation
// must be numerically invariant under column scaling because the columns of
// W and P converge to zero at different rates.
bool chol_scaled(int n, const double *G, double *R)
{
    std::vector<double> d(n);
    for (int i = 0; i < n; i++) {
        double g = G[i * n + i];
        if (!(g > 0.0) || !std::isfinite(g)) return false;
        d[i] = std::sqrt(g);
    }
    std::vector<double> H(size_t(n) * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            // symmetrise from the two triangles, then scale
            double g = 0.5 * (G[i * n + j] + G[j * n + i]);
            H[i * n + j] = g / (d[i] * d[j]);
        }
    // upper Cholesky Rh, one row at a time: row i of Rh from row i of H, then
    // its outer product taken off the trailing rows of H (the subtractions
    // of each entry in the same order as a dot product over k < i, with
    // contiguous rows)
    std::fill(R, R + size_t(n) * n, 0.0);
    for (int i = 0; i < n; i++) {
        const double s = H[i * n + i];
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        const double rii = std::sqrt(s);
        double *ri = R + size_t(i) * n;
        ri[i] = rii;
        for (int j = i + 1; j < n; j++) ri[j] = H[i * n + j] / rii;
        for (int j = i + 1; j < n; j++) {
            const double rj = ri[j];
            double *hj = H.data() + size_t(j) * n;
            for (int l = j; l < n; l++) hj[l] -= rj * ri[l];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = i; j < n; j++) R[i * n + j] *= d[j];
    return true;
}

// Inverse of an upper-triangular n x n matrix (row-major), by back
// substitution, one row of the inverse at a time from the last:
// Ri[i][:] = (e_i - sum_{k>i} R[i][k] Ri[k][:]) / R[i][i].
bool triu_inverse(int n, const double *R, double *Ri)
{
    std::fill(Ri, Ri + size_t(n) * n, 0.0);
    for (int i = n - 1; i >= 0; i--) {
        const double rii = R[i * n + i];
        if (rii == 0.0 || !std::isfinite(rii)) return false;
        double *out = Ri + size_t(i) * n;
        out[i] = 1.0;
        for (int k = i + 1; k < n; k++) {
            const double r = R[i * n + k];
            const double *rk = Ri + size_t(k) * n;
            for (int j = k; j < n; j++) out[j] -= r * rk[j];
        }
        for (int j = i; j < n; j++) out[j] /= rii;
    }
    return true;
}

namespace {

// Givens rotation (c, s) with [c s; -s c]^T [a; b] = [r; 0].
inline void givens(double a, double b, double &c, double &s)
{
    if (b == 0.0) {
        c = 1.0;
        s = 0.0;
    } else if (std::fabs(b) > std::fabs(a)) {
        double t = -a / b;
        s = 1.0 / std::sqrt(1.0 + t * t);
        c = s * t;
    } else {
        double t = -b / a;
        c = 1.0 / std::sqrt(1.0 + t * t);
        s = c * t;
    }
}

// Householder tridiagonalisation of the symmetric n x n matrix A (row-major,
// overwritten).  On return d (diagonal), e (e[i] = T[i][i+1]) and Qt with
// A = Q T Q^T stored as rows of Q^T (Qt[i*n + :] = column i of Q).
void tridiagonalize(int n, double *A, double *d, double *e, double *Qt)
{
    std::vector<double> v(n), p(n), w(n);
    for (int i = 0; i < n * n; i++) Qt[i] = 0.0;
    for (int i = 0; i < n; i++) Qt[i * n + i] = 1.0;
    for (int k = 0; k + 2 < n; k++) {
        // Householder vector for x = A[k+1:n][k]
        double alpha = 0.0;
        for (int i = k + 1; i < n; i++) alpha += A[i * n + k] * A[i * n + k];
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        double x0 = A[(k + 1) * n + k];
        if (x0 > 0) alpha = -alpha;                 // avoid cancellation: H x = alpha e1
        for (int i = 0; i < n; i++) v[i] = 0.0;
        v[k + 1] = x0 - alpha;
        for (int i = k + 2; i < n; i++) v[i] = A[i * n + k];
        double vnorm2 = 0.0;
        for (int i = k + 1; i < n; i++) vnorm2 += v[i] * v[i];
        if (vnorm2 == 0.0) continue;
        double beta = 2.0 / vnorm2;
        // p = beta A v on the trailing block, w = p - (beta/2)(p.v) v
        for (int i = k + 1; i < n; i++) {
            double s = 0.0;
            for (int j = k + 1; j < n; j++) s += A[i * n + j] * v[j];
            p[i] = beta * s;
        }
        double pv = 0.0;
        for (int i = k + 1; i < n; i++) pv += p[i] * v[i];
        for (int i = k + 1; i < n; i++) w[i] = p[i] - 0.5 * beta * pv * v[i];
        // A <- A - v w^T - w v^T on the trailing block
        for (int i = k + 1; i < n; i++)
            for (int j = k + 1; j < n; j++) A[i * n + j] -= v[i] * w[j] + w[i] * v[j];
        A[(k + 1) * n + k] = A[k * n + k + 1] = alpha;
        for (int i = k + 2; i < n; i++) A[i * n + k] = A[k * n + i] = 0.0;
        // Q <- Q H: column j of Q is row j of Qt; H = I - beta v v^T acts on
        // columns k+1..n-1, i.e. Qt rows: Qt[j][i] -= beta (sum_l Qt[l][i] v[l]) v[j]
        for (int i = 0; i < n; i++) p[i] = 0.0;
        for (int l = k + 1; l < n; l++) {
            const double vl = v[l];
            const double *ql = Qt + size_t(l) * n;
            for (int i = 0; i < n; i++) p[i] += ql[i] * vl;
        }
        for (int i = 0; i < n; i++) p[i] *= beta;
        for (int l = k + 1; l < n; l++) {
            const double vl = v[l];
            double *ql = Qt + size_t(l) * n;
            for (int i = 0; i < n; i++) ql[i] -= p[i] * vl;
        }
    }
    for (int i = 0; i < n; i++) d[i] = A[i * n + i];
    for (int i = 0; i + 1 < n; i++) e[i] = A[i * n + i + 1];
    if (n > 0) e[n - 1] = 0.0;
}

// Rows (a, b) <- (c a - s b, s a + c b).  Most of the eigensolver's time is
// spent here; the AVX2 clone (chosen at load time where the CPU has it)
// does the same operations per element, four at a time.
__attribute__((target_clones("avx2", "default"))) void rotate_rows(double *__restrict__ a, double *__restrict__ b,
                                                                    int n, double c, double s)
{
    for (int i = 0; i < n; i++) {
        const double u = a[i], t = b[i];
        a[i] = c * u - s * t;
        b[i] = s * u + c * t;
    }
}

// Implicit symmetric QR with Wilkinson shift on the tridiagonal (d, e);
// rotations are applied to the rows of Zt (the eigenvector rows).
bool tridiagonal_qr(int n, double *d, double *e, double *Zt)
{
    int h = n - 1;
    int guard = 0;
    while (h > 0) {
        // deflate negligible off-diagonals
        for (int i = 0; i < h; i++)
            if (std::fabs(e[i]) <= DBL_EPSILON * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
        if (e[h - 1] == 0.0) {
            h--;
            continue;
        }
        if (++guard > 60 * n) return false;
        int l = h - 1;
        while (l > 0 && e[l - 1] != 0.0) l--;
        // Wilkinson shift from the trailing 2x2 block of [l, h]
        double dd = 0.5 * (d[h - 1] - d[h]);
        double b2 = e[h - 1] * e[h - 1];
        double sg = dd >= 0.0 ? 1.0 : -1.0;
        double mu = d[h] - b2 / (dd + sg * std::sqrt(dd * dd + b2));
        double x = d[l] - mu, z = e[l];
        double bulge = 0.0;
        for (int k = l; k < h; k++) {
            double c, s;
            givens(x, z, c, s);
            if (k > l) {
                // the rotation zeroes the bulge T[k-1][k+1]
                e[k - 1] = c * e[k - 1] - s * bulge;
            }
            double a = d[k], b = e[k], dn = d[k + 1];
            d[k] = c * c * a - 2.0 * c * s * b + s * s * dn;
            e[k] = c * s * a + (c * c - s * s) * b - c * s * dn;
            d[k + 1] = s * s * a + 2.0 * c * s * b + c * c * dn;
            if (k + 1 < h) {
                bulge = -s * e[k + 1];
                e[k + 1] = c * e[k + 1];
                x = e[k];
                z = bulge;
            }
            rotate_rows(Zt + size_t(k) * n, Zt + size_t(k + 1) * n, n, c, s);
        }
    }
    return true;
}

}  // namespace

// Eigen-decomposition of the symmetric n x n matrix S (row-major, read only):
// ascending eigenvalues w and eigenvectors V (n x n row-major, column j is the
// eigenvector of w[j]).
bool sym_eig(int n, const double *S, double *w, double *V)
{
    std::vector<double> A(S, S + size_t(n) * n), e(n), Zt(size_t(n) * n), d(n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double x = S[i * n + j];
            if (!std::isfinite(x)) return false;
            A[i * n + j] = 0.5 * (x + S[j * n + i]);
        }
    tridiagonalize(n, A.data(), d.data(), e.data(), Zt.data());
    if (!tridiagonal_qr(n, d.data(), e.data(), Zt.data())) return false;
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
    for (int j = 0; j < n; j++) {
        w[j] = d[order[j]];
        const double *row = Zt.data() + size_t(order[j]) * n;
        for (int i = 0; i < n; i++) V[i * n + j] = row[i];
    }
    return true;
}

// Step 24: gramA C = gramB C Theta.  With gramB = R^T R (scale-invariant
// Cholesky), M = R^-T gramA R^-1, M Y = Y Theta and C = R^-1 Y, so that
// C^T gramB C = Y^T Y = I.
bool rayleigh_ritz(int n, int m, const double *gramA, const double *gramB, double *theta, double *C)
{
    std::vector<double> R(size_t(n) * n), Ri(size_t(n) * n), T1(size_t(n) * n), M(size_t(n) * n),
        w(n), Y(size_t(n) * n);
    if (!chol_scaled(n, gramB, R.data())) return false;
    if (!triu_inverse(n, R.data(), Ri.data())) return false;
    // T1 = gramA Ri (the symmetric part of gramA); the products run over
    // contiguous rows, each entry summed over k in increasing order
    for (int i = 0; i < n; i++) {
        double *t = T1.data() + size_t(i) * n;
        for (int k = 0; k < n; k++) {
            const double a = 0.5 * (gramA[i * n + k] + gramA[k * n + i]);
            const double *rk = Ri.data() + size_t(k) * n;
            for (int j = k; j < n; j++) t[j] += a * rk[j];
        }
    }
    // M = Ri^T T1
    for (int i = 0; i < n; i++) {
        double *mi = M.data() + size_t(i) * n;
        for (int k = 0; k <= i; k++) {
            const double r = Ri[k * n + i];
            const double *tk = T1.data() + size_t(k) * n;
            for (int j = 0; j < n; j++) mi[j] += r * tk[j];
        }
    }
    if (!sym_eig(n, M.data(), w.data(), Y.data())) return false;
    for (int j = 0; j < m; j++) theta[j] = w[j];
    // C = Ri Y[:, :m]
    for (int i = 0; i < n; i++) {
        double *ci = C + size_t(i) * m;
        for (int j = 0; j < m; j++) ci[j] = 0.0;
        for (int k = i; k < n; k++) {
            const double r = Ri[i * n + k];
            const double *yk = Y.data() + size_t(k) * n;
            for (int j = 0; j < m; j++) ci[j] += r * yk[j];
        }
    }
    return true;
}

}  // namespace lobpcg
