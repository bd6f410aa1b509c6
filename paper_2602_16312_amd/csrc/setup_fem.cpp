// Host setup, part 1: reference element, geometry, interior faces and the
// SIPDG cell/face blocks of A_0 = cM M + A (section 3: the forms a_h and m_h
// and the penalty defined after them; section 3.1 for cM).
//
// Readings shared with the rest of the library: the penalty term enters a_h
// with a plus sign (symmetric interior penalty), sigma = eta * mean(n^T D+ n,
// n^T D- n) pointwise with eta = c p(p+1) mean(|F|/|K+|, |F|/|K-|) (c = 1 is
// the paper's choice, c > 1 a safety factor for distorted cells) unless a
// fixed eta is given; boundary faces carry no terms (homogeneous Neumann);
// Gauss-Legendre rules with p+1 points per direction on cells and faces.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace dgmg {

static std::vector<double> gauss_lobatto_01(int p) {
    if (p == 1) return {0.0, 1.0};
    if (p == 2) return {0.0, 0.5, 1.0};
    if (p == 3) {
        const double s = std::sqrt(0.2);
        return {0.0, 0.5 * (1.0 - s), 0.5 * (1.0 + s), 1.0};
    }
    if (p == 4) {
        const double s = std::sqrt(3.0 / 7.0);
        return {0.0, 0.5 * (1.0 - s), 0.5, 0.5 * (1.0 + s), 1.0};
    }
    fail(DGMG_EUNSUPPORTED, "polynomial degree must be 1 to 4");
}

// n-point Gauss-Legendre rule on [0,1]: Newton iteration on P_n from the
// Chebyshev-like initial guesses, weights 2 / ((1 - x^2) P_n'(x)^2) on [-1,1].
static void gauss_legendre_01(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? z : p1;
            double pm = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? z : p1;
            double pm = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
        }
        // ascending order on [0,1]
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = (2/((1-z^2)dp^2)) / 2
    }
}

void lagrange1d(const std::vector<double>& t, double x, double* val, double* der) {
    const int n = (int)t.size();
    for (int j = 0; j < n; ++j) {
        double v = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != j) v *= (x - t[m]) / (t[j] - t[m]);
        val[j] = v;
        if (der) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) {
                if (k == j) continue;
                double term = 1.0 / (t[j] - t[k]);
                for (int m = 0; m < n; ++m)
                    if (m != j && m != k) term *= (x - t[m]) / (t[j] - t[m]);
                s += term;
            }
            der[j] = s;
        }
    }
}

void RefElement::init(int dim, int deg) {
    if (dim != 2 && dim != 3) fail(DGMG_EUNSUPPORTED, "dimension must be 2 or 3");
    d = dim;
    p = deg;
    q = p + 1;
    if (q > kMaxQ || (dim == 3 && p > 3)) fail(DGMG_EUNSUPPORTED, "polynomial degree must be 1 to 4 (2D) or 1 to 3 (3D)");
    nodes = gauss_lobatto_01(p);
    gauss_legendre_01(q, gx, gw);
    b = 1;
    for (int k = 0; k < d; ++k) b *= q;
    qc = b;
    cq_xi.assign((size_t)qc * d, 0.0);
    cq_w.assign(qc, 1.0);
    for (int iq = 0; iq < qc; ++iq) {
        int r = iq;
        for (int k = 0; k < d; ++k) {
            int a = r % q;
            r /= q;
            cq_xi[(size_t)iq * d + k] = gx[a];
            cq_w[iq] *= gw[a];
        }
    }
    cq_phi.assign((size_t)qc * b, 0.0);
    cq_dphi.assign((size_t)qc * b * d, 0.0);
    for (int iq = 0; iq < qc; ++iq)
        tensor_eval(*this, &cq_xi[(size_t)iq * d], &cq_phi[(size_t)iq * b],
                    &cq_dphi[(size_t)iq * b * d]);
}

void tensor_eval(const RefElement& re, const double* xi, double* phi, double* grad) {
    double v[3][kMaxQ], dv[3][kMaxQ];
    for (int k = 0; k < re.d; ++k) lagrange1d(re.nodes, xi[k], v[k], dv[k]);
    for (int i = 0; i < re.b; ++i) {
        int idx[3] = {0, 0, 0};
        int r = i;
        for (int k = 0; k < re.d; ++k) {
            idx[k] = r % re.q;
            r /= re.q;
        }
        double f = 1.0;
        for (int k = 0; k < re.d; ++k) f *= v[k][idx[k]];
        phi[i] = f;
        if (grad) {
            for (int k = 0; k < re.d; ++k) {
                double g = 1.0;
                for (int m = 0; m < re.d; ++m) g *= (m == k) ? dv[m][idx[m]] : v[m][idx[m]];
                grad[(size_t)i * re.d + k] = g;
            }
        }
    }
}

void cell_map(int d, const double* X, const double* xi, double* x, double* J, double* det,
              double* JinvT) {
    const int nc = 1 << d;
    for (int a = 0; a < d; ++a) {
        if (x) x[a] = 0.0;
        for (int k = 0; k < d; ++k) J[a * d + k] = 0.0;
    }
    for (int c = 0; c < nc; ++c) {
        double f[3], df[3];
        for (int k = 0; k < d; ++k) {
            int bit = (c >> k) & 1;
            f[k] = bit ? xi[k] : 1.0 - xi[k];
            df[k] = bit ? 1.0 : -1.0;
        }
        double psi = 1.0;
        for (int k = 0; k < d; ++k) psi *= f[k];
        for (int k = 0; k < d; ++k) {
            double g = df[k];
            for (int m = 0; m < d; ++m)
                if (m != k) g *= f[m];
            for (int a = 0; a < d; ++a) J[a * d + k] += X[c * d + a] * g;
        }
        if (x)
            for (int a = 0; a < d; ++a) x[a] += X[c * d + a] * psi;
    }
    if (d == 2) {
        double dt = J[0] * J[3] - J[1] * J[2];
        *det = dt;
        // J^-1 = [[J11, -J01], [-J10, J00]] / det; JinvT[a][k] = Jinv[k][a]
        JinvT[0] = J[3] / dt;
        JinvT[1] = -J[2] / dt;
        JinvT[2] = -J[1] / dt;
        JinvT[3] = J[0] / dt;
    } else {
        const double *r0 = J, *r1 = J + 3, *r2 = J + 6;
        double c00 = r1[1] * r2[2] - r1[2] * r2[1];
        double c01 = r1[2] * r2[0] - r1[0] * r2[2];
        double c02 = r1[0] * r2[1] - r1[1] * r2[0];
        double c10 = r0[2] * r2[1] - r0[1] * r2[2];
        double c11 = r0[0] * r2[2] - r0[2] * r2[0];
        double c12 = r0[1] * r2[0] - r0[0] * r2[1];
        double c20 = r0[1] * r1[2] - r0[2] * r1[1];
        double c21 = r0[2] * r1[0] - r0[0] * r1[2];
        double c22 = r0[0] * r1[1] - r0[1] * r1[0];
        double dt = r0[0] * c00 + r0[1] * c01 + r0[2] * c02;
        *det = dt;
        // inverse transpose = cofactor matrix / det
        JinvT[0] = c00 / dt; JinvT[1] = c01 / dt; JinvT[2] = c02 / dt;
        JinvT[3] = c10 / dt; JinvT[4] = c11 / dt; JinvT[5] = c12 / dt;
        JinvT[6] = c20 / dt; JinvT[7] = c21 / dt; JinvT[8] = c22 / dt;
    }
}

// ------------------------------------------------------------------ faces
Faces find_faces(const Hierarchy& h) {
    const int d = h.dim, nc = 1 << d, nfv = nc / 2;
    struct Rec {
        std::array<int64_t, 4> key;
        int64_t cell;
        int axis, side;
    };
    std::vector<Rec> recs;
    recs.reserve((size_t)h.n_cells * 2 * d);
    for (int64_t c = 0; c < h.n_cells; ++c) {
        const int64_t* cv = &h.cells[(size_t)c * nc];
        for (int k = 0; k < d; ++k)
            for (int s = 0; s < 2; ++s) {
                Rec r;
                r.key = {-1, -1, -1, -1};
                int m = 0;
                for (int corner = 0; corner < nc; ++corner)
                    if (((corner >> k) & 1) == s) r.key[m++] = cv[corner];
                std::sort(r.key.begin(), r.key.begin() + nfv);
                r.cell = c;
                r.axis = k;
                r.side = s;
                recs.push_back(r);
            }
    }
    std::sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) {
        if (a.key != b.key) return a.key < b.key;
        return a.cell < b.cell;
    });
    Faces F;
    size_t i = 0;
    while (i < recs.size()) {
        size_t j = i + 1;
        while (j < recs.size() && recs[j].key == recs[i].key) ++j;
        if (j - i > 2) fail(DGMG_EINVAL, "a face is shared by more than two cells");
        if (j - i == 2) {
            const Rec* a = &recs[i];
            const Rec* b = &recs[i + 1];
            if (a->side == 0) std::swap(a, b);
            if (a->axis != b->axis || a->side != 1 || b->side != 0)
                fail(DGMG_EUNSUPPORTED, "face neighbours are not consistently oriented");
            // identical tangential order of the shared corners
            const int64_t* ca = &h.cells[(size_t)a->cell * nc];
            const int64_t* cb = &h.cells[(size_t)b->cell * nc];
            for (int corner = 0; corner < nc; ++corner)
                if (((corner >> a->axis) & 1) == 1) {
                    int partner = corner & ~(1 << a->axis);
                    if (ca[corner] != cb[partner])
                        fail(DGMG_EUNSUPPORTED, "face vertex order differs between neighbours");
                }
            F.plus.push_back(a->cell);
            F.minus.push_back(b->cell);
            F.axis.push_back(a->axis);
        }
        i = j;
    }
    // order faces by (plus cell, axis) so a cell's own faces are contiguous
    std::vector<size_t> ord(F.plus.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
    std::sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
        if (F.plus[x] != F.plus[y]) return F.plus[x] < F.plus[y];
        return F.axis[x] < F.axis[y];
    });
    Faces G;
    G.plus.resize(ord.size());
    G.minus.resize(ord.size());
    G.axis.resize(ord.size());
    for (size_t k = 0; k < ord.size(); ++k) {
        G.plus[k] = F.plus[ord[k]];
        G.minus[k] = F.minus[ord[k]];
        G.axis[k] = F.axis[ord[k]];
    }
    return G;
}

// ------------------------------------------------------------- assembly
void FaceRef::init(const RefElement& re) {
    const int d = re.d, b = re.b;
    qf = b / re.q;
    xi_p.assign((size_t)d * qf * d, 0.0);
    xi_m.assign((size_t)d * qf * d, 0.0);
    w.assign((size_t)d * qf, 0.0);
    phi_p.assign((size_t)d * qf * b, 0.0);
    phi_m.assign((size_t)d * qf * b, 0.0);
    g_p.assign((size_t)d * qf * b * d, 0.0);
    g_m.assign((size_t)d * qf * b * d, 0.0);
    for (int ax = 0; ax < d; ++ax) {
        for (int iq = 0; iq < qf; ++iq) {
            double xp[3], xm[3], wt = 1.0;
            int r = iq;
            for (int k = 0; k < d; ++k) {
                if (k == ax) {
                    xp[k] = 1.0;
                    xm[k] = 0.0;
                } else {
                    int a = r % re.q;
                    r /= re.q;
                    xp[k] = xm[k] = re.gx[a];
                    wt *= re.gw[a];
                }
            }
            size_t o = (size_t)ax * qf + iq;
            for (int k = 0; k < d; ++k) {
                xi_p[o * d + k] = xp[k];
                xi_m[o * d + k] = xm[k];
            }
            w[o] = wt;
            tensor_eval(re, xp, &phi_p[o * b], &g_p[o * b * d]);
            tensor_eval(re, xm, &phi_m[o * b], &g_m[o * b * d]);
        }
    }
}

static void unpack_D(int d, const double* Dp, double s, double* D) {
    if (d == 2) {
        D[0] = s * Dp[0]; D[1] = s * Dp[1];
        D[2] = s * Dp[1]; D[3] = s * Dp[2];
    } else {
        D[0] = s * Dp[0]; D[1] = s * Dp[1]; D[2] = s * Dp[2];
        D[3] = s * Dp[1]; D[4] = s * Dp[3]; D[5] = s * Dp[4];
        D[6] = s * Dp[2]; D[7] = s * Dp[4]; D[8] = s * Dp[5];
    }
}

static void corners_of(const Hierarchy& h, int64_t c, double* X) {
    const int d = h.dim, nc = 1 << d;
    for (int k = 0; k < nc; ++k) {
        int64_t v = h.cells[(size_t)c * nc + k];
        for (int a = 0; a < d; ++a) X[k * d + a] = h.xyz[(size_t)v * d + a];
    }
}

void assemble_fine(const Hierarchy& h, const Faces& F, const RefElement& re,
                   const dgmg_disc& disc, const dgmg_physics& ph, double cM, BlockOp& A0,
                   std::vector<double>& mass, AdjointBlocks* adj) {
    const int d = re.d, b = re.b, bb = b * b, symn = d * (d + 1) / 2;
    const int64_t n = h.n_cells;
    A0.n = n;
    A0.b = b;
    A0.diag.assign((size_t)n * bb, 0.0);
    mass.assign((size_t)n * bb, 0.0);
    std::vector<double> vol(n, 0.0);
    if (adj) {
        adj->S.assign((size_t)n * bb, 0.0);
        adj->X.assign((size_t)F.plus.size() * 2 * 4 * bb, 0.0);
    }
    int bad = 0;

#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t c = 0; c < n; ++c) {
        double X[24], D[9], J[9], det, JiT[9];
        corners_of(h, c, X);
        const double sc = ph.cell_scale ? ph.cell_scale[c] : 1.0;
        unpack_D(d, &ph.D_cell[(size_t)c * symn], 1.0, D);   // unscaled: S_K is linear in D
        std::vector<double> G((size_t)b * d), DG((size_t)b * d), Sun((size_t)bb, 0.0);
        double* Md = &mass[(size_t)c * bb];
        double* Ad = &A0.diag[(size_t)c * bb];
        double v = 0.0;
        for (int iq = 0; iq < re.qc; ++iq) {
            cell_map(d, X, &re.cq_xi[(size_t)iq * d], nullptr, J, &det, JiT);
            if (!(det > 0.0)) ++bad;
            const double wd = re.cq_w[iq] * std::fabs(det);
            v += wd;
            const double* phi = &re.cq_phi[(size_t)iq * b];
            const double* gr = &re.cq_dphi[(size_t)iq * b * d];
            for (int i = 0; i < b; ++i)
                for (int a = 0; a < d; ++a) {
                    double s = 0.0;
                    for (int k = 0; k < d; ++k) s += JiT[a * d + k] * gr[i * d + k];
                    G[i * d + a] = s;
                }
            for (int i = 0; i < b; ++i)
                for (int a = 0; a < d; ++a) {
                    double s = 0.0;
                    for (int k = 0; k < d; ++k) s += D[a * d + k] * G[i * d + k];
                    DG[i * d + a] = s;
                }
            for (int i = 0; i < b; ++i)
                for (int j = 0; j < b; ++j) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) s += G[i * d + a] * DG[j * d + a];
                    Md[i * b + j] += wd * phi[i] * phi[j];
                    Sun[i * b + j] += wd * s;
                }
        }
        vol[c] = v;
        for (int k = 0; k < bb; ++k) Ad[k] = sc * Sun[k] + cM * Md[k];
        if (adj) std::copy(Sun.begin(), Sun.end(), adj->S.begin() + (size_t)c * bb);
    }
    if (bad) fail(DGMG_EINVAL, "non-positive Jacobian determinant in the mesh");

    // reference data of the face rule for each axis
    FaceRef fr;
    fr.init(re);
    const int qf = fr.qf;
    const int64_t nf = (int64_t)F.plus.size();
    A0.nf = nf;
    A0.fc.resize((size_t)nf * 2);
    A0.fblk.assign((size_t)nf * bb, 0.0);
    const std::vector<double>&fxi_p = fr.xi_p, &fxi_m = fr.xi_m, &fw = fr.w;
    const std::vector<double>&fphi_p = fr.phi_p, &fphi_m = fr.phi_m, &fg_p = fr.g_p, &fg_m = fr.g_m;
    const int B2 = 2 * b;
    // local 2b x 2b matrix of the face terms of a_h over [K+ DoFs, K- DoFs]
    // for the given (already scaled) tensors of the two sides
    auto face_local = [&](int64_t f, const double* Dp, const double* Dm, double* L) {
        const int64_t cp = F.plus[f], cm = F.minus[f];
        const int ax = F.axis[f];
        double Xp[24], Xm[24], J[9], detp, detm, JiTp[9], JiTm[9];
        corners_of(h, cp, Xp);
        corners_of(h, cm, Xm);
        std::fill(L, L + (size_t)B2 * B2, 0.0);
        // |F| first (needed by the paper's penalty)
        std::vector<double> nrmv((size_t)qf * d), dS(qf);
        double area = 0.0;
        for (int iq = 0; iq < qf; ++iq) {
            size_t o = (size_t)ax * qf + iq;
            cell_map(d, Xp, &fxi_p[o * d], nullptr, J, &detp, JiTp);
            double nv[3], nn = 0.0;
            for (int a = 0; a < d; ++a) {
                nv[a] = JiTp[a * d + ax];
                nn += nv[a] * nv[a];
            }
            nn = std::sqrt(nn);
            for (int a = 0; a < d; ++a) nrmv[(size_t)iq * d + a] = nv[a] / nn;
            dS[iq] = fw[o] * std::fabs(detp) * nn;
            area += dS[iq];
        }
        const double cpen = disc.eta > 0.0 ? disc.eta : 1.0;
        double eta = disc.penalty_mode == DGMG_PENALTY_FIXED
                         ? disc.eta
                         : cpen * re.p * (re.p + 1) * 0.5 * (area / vol[cp] + area / vol[cm]);
        std::vector<double> jump(B2), flux(B2);
        for (int iq = 0; iq < qf; ++iq) {
            size_t o = (size_t)ax * qf + iq;
            cell_map(d, Xp, &fxi_p[o * d], nullptr, J, &detp, JiTp);
            cell_map(d, Xm, &fxi_m[o * d], nullptr, J, &detm, JiTm);
            const double* nv = &nrmv[(size_t)iq * d];
            double Dnp[3], Dnm[3], nDn = 0.0;
            for (int a = 0; a < d; ++a) {
                Dnp[a] = Dnm[a] = 0.0;
                for (int k = 0; k < d; ++k) {
                    Dnp[a] += Dp[a * d + k] * nv[k];
                    Dnm[a] += Dm[a * d + k] * nv[k];
                }
            }
            for (int a = 0; a < d; ++a) nDn += 0.5 * nv[a] * (Dnp[a] + Dnm[a]);
            const double sig = eta * nDn;
            for (int i = 0; i < b; ++i) {
                const double* gp = &fg_p[(o * b + i) * d];
                const double* gm = &fg_m[(o * b + i) * d];
                double fp = 0.0, fm = 0.0;
                for (int a = 0; a < d; ++a) {
                    double Gp = 0.0, Gm = 0.0;
                    for (int k = 0; k < d; ++k) {
                        Gp += JiTp[a * d + k] * gp[k];
                        Gm += JiTm[a * d + k] * gm[k];
                    }
                    fp += Gp * Dnp[a];
                    fm += Gm * Dnm[a];
                }
                jump[i] = fphi_p[o * b + i];
                jump[b + i] = -fphi_m[o * b + i];
                flux[i] = fp;
                flux[b + i] = fm;
            }
            const double w = dS[iq];
            for (int I = 0; I < B2; ++I)
                for (int Jx = 0; Jx < B2; ++Jx)
                    L[I * B2 + Jx] += w * (-0.5 * jump[I] * flux[Jx] - 0.5 * flux[I] * jump[Jx] +
                                           sig * jump[I] * jump[Jx]);
        }
    };
    const int64_t chunk = 16384;
    std::vector<double> loc((size_t)chunk * B2 * B2);
    for (int64_t f0 = 0; f0 < nf; f0 += chunk) {
        const int64_t f1 = std::min(nf, f0 + chunk);
#pragma omp parallel for schedule(static)
        for (int64_t f = f0; f < f1; ++f) {
            const int64_t cp = F.plus[f], cm = F.minus[f];
            double Dp[9], Dm[9], Z[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            unpack_D(d, &ph.D_cell[(size_t)cp * symn], ph.cell_scale ? ph.cell_scale[cp] : 1.0, Dp);
            unpack_D(d, &ph.D_cell[(size_t)cm * symn], ph.cell_scale ? ph.cell_scale[cm] : 1.0, Dm);
            face_local(f, Dp, Dm, &loc[(size_t)(f - f0) * B2 * B2]);
            if (adj) {
                // side-split derivative blocks with the unscaled tensors
                double Up[9], Um[9];
                unpack_D(d, &ph.D_cell[(size_t)cp * symn], 1.0, Up);
                unpack_D(d, &ph.D_cell[(size_t)cm * symn], 1.0, Um);
                face_local(f, Up, Z, &adj->X[(size_t)f * 2 * B2 * B2]);
                face_local(f, Z, Um, &adj->X[((size_t)f * 2 + 1) * B2 * B2]);
            }
        }
        // accumulate serially (cells shared between faces of a chunk)
        for (int64_t f = f0; f < f1; ++f) {
            const int64_t cp = F.plus[f], cm = F.minus[f];
            const double* L = &loc[(size_t)(f - f0) * B2 * B2];
            double* Dpl = &A0.diag[(size_t)cp * bb];
            double* Dmi = &A0.diag[(size_t)cm * bb];
            double* Fb = &A0.fblk[(size_t)f * bb];
            for (int i = 0; i < b; ++i)
                for (int j = 0; j < b; ++j) {
                    Dpl[i * b + j] += L[i * B2 + j];
                    Dmi[i * b + j] += L[(b + i) * B2 + (b + j)];
                    Fb[i * b + j] = L[i * B2 + (b + j)];
                }
            A0.fc[(size_t)f * 2] = cp;
            A0.fc[(size_t)f * 2 + 1] = cm;
        }
    }
}

}  // namespace dgmg
