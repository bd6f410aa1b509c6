// Host setup, part 2: agglomerated hierarchy, bounding-box prolongation
// blocks, blockwise Galerkin products, Lanczos eigenvalue estimates and the
// dense coarse factorisation (section 4; section 5.1 with eq.
// inherited_matrices and Algorithm 3; section 6 for the smoother set-up).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace dgmg {

// Level-l id of every fine cell.
static std::vector<int64_t> fine_to_level(const Hierarchy& h, int level) {
    std::vector<int64_t> id(h.n_cells);
    std::iota(id.begin(), id.end(), 0);
    for (int l = 0; l < level; ++l)
        for (auto& v : id) v = h.parent[l][v];
    return id;
}

void level_boxes(const Hierarchy& h, int level, std::vector<double>& lo, std::vector<double>& hi) {
    const int d = h.dim, nc = 1 << d;
    const int64_t n = h.n_ent[level];
    lo.assign((size_t)n * d, INFINITY);
    hi.assign((size_t)n * d, -INFINITY);
    std::vector<int64_t> id = fine_to_level(h, level);
    for (int64_t c = 0; c < h.n_cells; ++c) {
        int64_t K = id[c];
        for (int k = 0; k < nc; ++k) {
            int64_t v = h.cells[(size_t)c * nc + k];
            for (int a = 0; a < d; ++a) {
                double x = h.xyz[(size_t)v * d + a];
                lo[(size_t)K * d + a] = std::min(lo[(size_t)K * d + a], x);
                hi[(size_t)K * d + a] = std::max(hi[(size_t)K * d + a], x);
            }
        }
    }
}

// P_e[i][j] = l^K_j(x_i): coarse tensor Lagrange basis on the parent's box,
// evaluated at the physical position of fine node i (the image of the GL
// reference node on level 0, the GL node of the child's box above).
void prolongation_blocks(const Hierarchy& h, const RefElement& re, int level,
                         const std::vector<double>& lo_l, const std::vector<double>& hi_l,
                         const std::vector<double>& lo_c, const std::vector<double>& hi_c,
                         std::vector<double>& P) {
    const int d = re.d, b = re.b, q = re.q, nc = 1 << d;
    const int64_t n = h.n_ent[level];
    P.assign((size_t)n * b * b, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
        const int64_t K = h.parent[level][e];
        double X[24];
        if (level == 0)
            for (int k = 0; k < nc; ++k) {
                int64_t v = h.cells[(size_t)e * nc + k];
                for (int a = 0; a < d; ++a) X[k * d + a] = h.xyz[(size_t)v * d + a];
            }
        for (int i = 0; i < b; ++i) {
            double xi[3], x[3];
            int r = i;
            for (int k = 0; k < d; ++k) {
                xi[k] = re.nodes[r % q];
                r /= q;
            }
            if (level == 0) {
                double J[9], det, JiT[9];
                cell_map(d, X, xi, x, J, &det, JiT);
            } else {
                for (int k = 0; k < d; ++k)
                    x[k] = lo_l[(size_t)e * d + k] + xi[k] * (hi_l[(size_t)e * d + k] - lo_l[(size_t)e * d + k]);
            }
            double l1[3][kMaxQ];
            for (int k = 0; k < d; ++k) {
                const double a = lo_c[(size_t)K * d + k], w = hi_c[(size_t)K * d + k] - a;
                lagrange1d(re.nodes, (x[k] - a) / w, l1[k], nullptr);
            }
            for (int j = 0; j < b; ++j) {
                double v = 1.0;
                int rj = j;
                for (int k = 0; k < d; ++k) {
                    v *= l1[k][rj % q];
                    rj /= q;
                }
                P[((size_t)e * b + i) * b + j] = v;
            }
        }
    }
}

// C = A^T B for b x b row-major blocks (accumulating into C when acc)
static void atb(int b, const double* A, const double* B, double* C) {
    for (int i = 0; i < b * b; ++i) C[i] = 0.0;
    for (int k = 0; k < b; ++k)
        for (int i = 0; i < b; ++i) {
            const double a = A[k * b + i];
            for (int j = 0; j < b; ++j) C[i * b + j] += a * B[k * b + j];
        }
}
static void ab(int b, const double* A, const double* B, double* C) {
    for (int i = 0; i < b * b; ++i) C[i] = 0.0;
    for (int i = 0; i < b; ++i)
        for (int k = 0; k < b; ++k) {
            const double a = A[i * b + k];
            for (int j = 0; j < b; ++j) C[i * b + j] += a * B[k * b + j];
        }
}

// Integer structure of the blockwise A_{l+1} = P^T A_l P.  A coarse cell
// block sums P_e^T A_ee P_e over its children (ascending e), then the face
// terms between two of its children (ascending f); a coarse face block sums
// P_{e+}^T A_f P_{e-} over the fine faces joining two different agglomerates
// (ascending f), stored with plus = smaller coarse id.
void galerkin_plan(const BlockOp& A, const std::vector<int64_t>& parent, int64_t nC, BlockOp& Ac,
                   GalerkinPlan& plan) {
    Ac.n = nC;
    Ac.b = A.b;
    std::vector<int64_t> key(A.nf);
    for (int64_t f = 0; f < A.nf; ++f) {
        int64_t Kp = parent[A.fc[2 * f]], Km = parent[A.fc[2 * f + 1]];
        key[f] = (Kp == Km) ? -1 : std::min(Kp, Km) * nC + std::max(Kp, Km);
    }
    std::vector<int64_t> ukeys;
    for (auto k : key)
        if (k >= 0) ukeys.push_back(k);
    std::sort(ukeys.begin(), ukeys.end());
    ukeys.erase(std::unique(ukeys.begin(), ukeys.end()), ukeys.end());
    Ac.nf = (int64_t)ukeys.size();
    Ac.fc.resize((size_t)Ac.nf * 2);
    for (int64_t g = 0; g < Ac.nf; ++g) {
        Ac.fc[2 * g] = ukeys[g] / nC;
        Ac.fc[2 * g + 1] = ukeys[g] % nC;
    }
    // target entity of every fine cell and face
    std::vector<int64_t> tf(A.nf);
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < A.nf; ++f)
        tf[f] = key[f] < 0 ? parent[A.fc[2 * f]]
                           : nC + (std::lower_bound(ukeys.begin(), ukeys.end(), key[f]) - ukeys.begin());
    const int64_t nt = nC + Ac.nf;
    plan.ptr.assign(nt + 1, 0);
    for (int64_t e = 0; e < A.n; ++e) plan.ptr[parent[e] + 1]++;
    for (int64_t f = 0; f < A.nf; ++f) plan.ptr[tf[f] + 1]++;
    for (int64_t t = 0; t < nt; ++t) plan.ptr[t + 1] += plan.ptr[t];
    plan.item.resize(plan.ptr[nt]);
    std::vector<int64_t> pos(plan.ptr.begin(), plan.ptr.end() - 1);
    for (int64_t e = 0; e < A.n; ++e) plan.item[pos[parent[e]]++] = e << 2;
    for (int64_t f = 0; f < A.nf; ++f) {
        const int64_t Kp = parent[A.fc[2 * f]], Km = parent[A.fc[2 * f + 1]];
        const int mode = Kp == Km ? 3 : (Kp < Km ? 1 : 2);
        plan.item[pos[tf[f]]++] = (f << 2) | mode;
    }
}

void galerkin(const BlockOp& A, const std::vector<double>& P, const std::vector<int64_t>& parent,
              int64_t nC, BlockOp& Ac) {
    GalerkinPlan plan;
    galerkin_plan(A, parent, nC, Ac, plan);
    const int b = A.b, bb = b * b;
    Ac.diag.assign((size_t)nC * bb, 0.0);
    Ac.fblk.assign((size_t)Ac.nf * bb, 0.0);
    const int64_t nt = nC + Ac.nf;
#pragma omp parallel
    {
        std::vector<double> t1(bb), t(bb);
#pragma omp for schedule(dynamic, 16)
        for (int64_t u = 0; u < nt; ++u) {
            double* out = u < nC ? &Ac.diag[(size_t)u * bb] : &Ac.fblk[(size_t)(u - nC) * bb];
            for (int64_t it = plan.ptr[u]; it < plan.ptr[u + 1]; ++it) {
                const int64_t src = plan.item[it] >> 2;
                const int mode = (int)(plan.item[it] & 3);
                const double* X = mode == 0 ? &A.diag[(size_t)src * bb] : &A.fblk[(size_t)src * bb];
                const int64_t ea = mode == 0 ? src : A.fc[2 * src];
                const int64_t ec = mode == 0 ? src : A.fc[2 * src + 1];
                ab(b, X, &P[(size_t)ec * bb], t1.data());
                atb(b, &P[(size_t)ea * bb], t1.data(), t.data());
                if (mode <= 1)
                    for (int k = 0; k < bb; ++k) out[k] += t[k];
                else if (mode == 2)
                    for (int i = 0; i < b; ++i)
                        for (int j = 0; j < b; ++j) out[i * b + j] += t[j * b + i];
                else
                    for (int i = 0; i < b; ++i)
                        for (int j = 0; j < b; ++j) out[i * b + j] += t[i * b + j] + t[j * b + i];
            }
        }
    }
}

// y = A x with a per-cell gather over the cell's faces (parallel, no races).
struct CellFaces {
    std::vector<int64_t> ptr, code;   // code = face << 1 | (cell is the minus side)
};
static CellFaces cell_faces(const BlockOp& A) {
    CellFaces C;
    cell_face_lists(A, C.ptr, C.code);
    return C;
}
void cell_face_lists(const BlockOp& A, std::vector<int64_t>& ptr, std::vector<int64_t>& code) {
    ptr.assign(A.n + 1, 0);
    for (int64_t f = 0; f < A.nf; ++f) {
        ptr[A.fc[2 * f] + 1]++;
        ptr[A.fc[2 * f + 1] + 1]++;
    }
    for (int64_t K = 0; K < A.n; ++K) ptr[K + 1] += ptr[K];
    code.resize(ptr[A.n]);
    std::vector<int64_t> pos(ptr.begin(), ptr.end() - 1);
    for (int64_t f = 0; f < A.nf; ++f) {
        code[pos[A.fc[2 * f]]++] = f << 1;
        code[pos[A.fc[2 * f + 1]]++] = (f << 1) | 1;
    }
}

static void apply_with(const BlockOp& A, const CellFaces& C, const double* x, double* y) {
    const int b = A.b, bb = b * b;
#pragma omp parallel for schedule(static)
    for (int64_t K = 0; K < A.n; ++K) {
        const double* D = &A.diag[(size_t)K * bb];
        for (int i = 0; i < b; ++i) {
            double s = 0.0;
            for (int j = 0; j < b; ++j) s += D[i * b + j] * x[K * b + j];
            y[K * b + i] = s;
        }
        for (int64_t e = C.ptr[K]; e < C.ptr[K + 1]; ++e) {
            const int64_t f = C.code[e] >> 1;
            const bool minus = (C.code[e] & 1) != 0;
            const int64_t nb = minus ? A.fc[2 * f] : A.fc[2 * f + 1];
            const double* F = &A.fblk[(size_t)f * bb];
            for (int i = 0; i < b; ++i) {
                double s = 0.0;
                if (!minus)
                    for (int j = 0; j < b; ++j) s += F[i * b + j] * x[nb * b + j];
                else
                    for (int j = 0; j < b; ++j) s += F[j * b + i] * x[nb * b + j];
                y[K * b + i] += s;
            }
        }
    }
}

void host_apply(const BlockOp& A, const double* x, double* y) { apply_with(A, cell_faces(A), x, y); }

// Largest eigenvalue of a symmetric tridiagonal matrix by Sturm-sequence
// bisection (count of eigenvalues below a shift).
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& bt) {
    const int m = (int)a.size();
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < m; ++i) {
        double r = (i > 0 ? std::fabs(bt[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(bt[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto count_below = [&](double s) {
        int cnt = 0;
        double q = 1.0;
        for (int i = 0; i < m; ++i) {
            double off = (i > 0) ? bt[i - 1] * bt[i - 1] : 0.0;
            q = a[i] - s - (i > 0 ? off / q : 0.0);
            if (q == 0.0) q = -1e-300;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (count_below(mid) >= m) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

void lanczos_start(int64_t n, std::vector<double>& v) {
    v.resize(n);
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = ((double)i + 1.0) * 0.6180339887498949;
        v[i] = t - std::floor(t) - 0.5;
        nrm += v[i] * v[i];
    }
    nrm = std::sqrt(nrm);
    for (auto& x : v) x /= nrm;
}

// Cell-block Jacobi: the Cholesky factor L_K (lower, row-major) of every
// diagonal block D_K and the inverse D_K^-1 = L_K^-T L_K^-1 (computed in its
// lower triangle and mirrored, so exactly symmetric).  A pivot <= 0 fails
// with DGMG_ENOTSPD.
void cell_block_factors(const BlockOp& A, std::vector<double>& Lc, std::vector<double>& Dinv) {
    const int b = A.b;
    const size_t bb = (size_t)b * b;
    Lc.assign(A.n * bb, 0.0);
    Dinv.assign(A.n * bb, 0.0);
    bool bad = false;
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (int64_t K = 0; K < A.n; ++K) {
        const double* D = &A.diag[K * bb];
        double* L = &Lc[K * bb];
        for (int j = 0; j < b && !bad; ++j) {
            double d = D[j * b + j];
            for (int k = 0; k < j; ++k) d -= L[j * b + k] * L[j * b + k];
            if (!(d > 0.0)) {
                bad = true;
                break;
            }
            L[j * b + j] = std::sqrt(d);
            for (int i = j + 1; i < b; ++i) {
                double v = D[i * b + j];
                for (int k = 0; k < j; ++k) v -= L[i * b + k] * L[j * b + k];
                L[i * b + j] = v / L[j * b + j];
            }
        }
        if (bad) continue;
        // columns of L^-1 by forward substitution, then D^-1 = L^-T L^-1
        std::vector<double> Li(bb, 0.0);
        for (int c = 0; c < b; ++c)
            for (int i = c; i < b; ++i) {
                double v = i == c ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) v -= L[i * b + k] * Li[k * b + c];
                Li[i * b + c] = v / L[i * b + i];
            }
        double* Z = &Dinv[K * bb];
        for (int i = 0; i < b; ++i)
            for (int j = 0; j <= i; ++j) {
                double v = 0.0;
                for (int k = i; k < b; ++k) v += Li[k * b + i] * Li[k * b + j];
                Z[i * b + j] = v;
                Z[j * b + i] = v;
            }
    }
    if (bad) fail(DGMG_ENOTSPD, "a diagonal cell block is not positive definite");
}

// m Lanczos steps on S A S^T without reorthogonalisation, S = D^-1/2 (point
// Jacobi) or S = L^-1 with D_K = L_K L_K^T per cell (cell-block Jacobi, chol
// given); start vector frac((i+1) * golden ratio conjugate) - 1/2, early stop
// when the next beta falls below 1e-14; returns the largest Ritz value.
double lanczos_theta_max(const BlockOp& A, int steps, const std::vector<double>* chol) {
    const int b = A.b;
    const size_t bb = (size_t)b * b;
    const int64_t n = A.n * b;
    std::vector<double> s(n), v(n), vp(n, 0.0), w(n), tmp(n);
    for (int64_t K = 0; K < A.n; ++K)
        for (int i = 0; i < b; ++i) s[K * b + i] = 1.0 / std::sqrt(A.diag[((size_t)K * b + i) * b + i]);
    // y = S^T x and y = S x (in place), per cell
    auto scale_t = [&](const double* x, double* y) {
        if (!chol) {
            for (int64_t i = 0; i < n; ++i) y[i] = s[i] * x[i];
            return;
        }
#pragma omp parallel for schedule(static)
        for (int64_t K = 0; K < A.n; ++K) {     // back substitution with L_K^T
            const double* L = &(*chol)[K * bb];
            for (int i = b - 1; i >= 0; --i) {
                double t = x[K * b + i];
                for (int k = i + 1; k < b; ++k) t -= L[k * b + i] * y[K * b + k];
                y[K * b + i] = t / L[i * b + i];
            }
        }
    };
    auto scale = [&](double* x) {
        if (!chol) {
            for (int64_t i = 0; i < n; ++i) x[i] *= s[i];
            return;
        }
#pragma omp parallel for schedule(static)
        for (int64_t K = 0; K < A.n; ++K) {     // forward substitution with L_K
            const double* L = &(*chol)[K * bb];
            for (int i = 0; i < b; ++i) {
                double t = x[K * b + i];
                for (int k = 0; k < i; ++k) t -= L[i * b + k] * x[K * b + k];
                x[K * b + i] = t / L[i * b + i];
            }
        }
    };
    lanczos_start(n, v);
    std::vector<double> al, be;
    double beta = 0.0;
    const int64_t mmax = std::min<int64_t>(steps, n);
    const CellFaces C = cell_faces(A);
    for (int64_t j = 0; j < mmax; ++j) {
        scale_t(v.data(), tmp.data());
        apply_with(A, C, tmp.data(), w.data());
        scale(w.data());
        double a = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            w[i] = w[i] - beta * vp[i];
            a += w[i] * v[i];
        }
        double bn = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            w[i] -= a * v[i];
            bn += w[i] * w[i];
        }
        al.push_back(a);
        beta = std::sqrt(bn);
        if (beta < 1e-14 || j == mmax - 1) break;
        be.push_back(beta);
        for (int64_t i = 0; i < n; ++i) {
            vp[i] = v[i];
            v[i] = w[i] / beta;
        }
    }
    be.resize(al.size() > 0 ? al.size() - 1 : 0);
    if (al.size() == 1) return al[0];
    return tridiag_max_eig(al, be);
}

void dense_from_blocks(const BlockOp& A, std::vector<double>& M) {
    const int b = A.b;
    const int64_t n = A.n * b;
    M.assign((size_t)n * n, 0.0);
    for (int64_t K = 0; K < A.n; ++K)
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j)
                M[(size_t)(K * b + i) * n + K * b + j] = A.diag[((size_t)K * b + i) * b + j];
    for (int64_t f = 0; f < A.nf; ++f) {
        const int64_t p = A.fc[2 * f], m = A.fc[2 * f + 1];
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
                double v = A.fblk[((size_t)f * b + i) * b + j];
                M[(size_t)(p * b + i) * n + m * b + j] += v;
                M[(size_t)(m * b + j) * n + p * b + i] += v;
            }
    }
}

// Row-major dense SPD matrix -> its inverse, via the lower Cholesky factor L
// (A = L L^T), X = L^-1 by forward substitution, A^-1 = X^T X.
void cholesky_inverse(std::vector<double>& a, int64_t n) {
    for (int64_t j = 0; j < n; ++j) {
        double* rj = &a[(size_t)j * n];
        double s = rj[j];
        for (int64_t k = 0; k < j; ++k) s -= rj[k] * rj[k];
        if (!(s > 0.0)) fail(DGMG_ENOTSPD, "coarse operator is not positive definite");
        const double ljj = std::sqrt(s);
        rj[j] = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            double* ri = &a[(size_t)i * n];
            double t = ri[j];
            for (int64_t k = 0; k < j; ++k) t -= ri[k] * rj[k];
            ri[j] = t / ljj;
        }
    }
    // X = L^-1 (lower), stored transposed as Xt[j][i] = X[i][j] for row access
    std::vector<double> Xt((size_t)n * n, 0.0);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < n; ++j) {
        double* x = &Xt[(size_t)j * n];   // column j of X
        x[j] = 1.0 / a[(size_t)j * n + j];
        for (int64_t i = j + 1; i < n; ++i) {
            const double* ri = &a[(size_t)i * n];
            double t = 0.0;
            for (int64_t k = j; k < i; ++k) t -= ri[k] * x[k];
            x[i] = t / ri[i];
        }
    }
    // A^-1[i][j] = sum_k X[k][i] X[k][j] = dot(column i, column j), k >= max(i,j)
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i) {
        const double* ci = &Xt[(size_t)i * n];
        for (int64_t j = 0; j <= i; ++j) {
            const double* cj = &Xt[(size_t)j * n];
            double t = 0.0;
            for (int64_t k = i; k < n; ++k) t += ci[k] * cj[k];
            a[(size_t)i * n + j] = t;
            a[(size_t)j * n + i] = t;
        }
    }
}

}  // namespace dgmg
