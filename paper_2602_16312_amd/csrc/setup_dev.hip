// Device part of the set-up: the fine SIPDG operator and mass blocks
// (section 3 and eq. fully_discrete), the prolongation blocks (section 5.1,
// tensor Lagrange bases on the agglomerates' bounding boxes), the blockwise
// Galerkin products A_{l+1} = P^T A_l P (section 5.1, eq.
// inherited_matrices) and the Lanczos estimate of the largest eigenvalue of
// D^-1 A_l that sets the Chebyshev interval (section 6).  The host supplies
// the integer structure (face lists, coarse face lists and the ordered
// contribution lists of every coarse block) and the reference-element
// tables; every floating-point operation of these phases runs here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.hpp"

namespace dgmg {
namespace {

#define DSCHK(expr)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            fail(DGMG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

constexpr int kSW = 256;   // threads per workgroup of the vector kernels

// ------------------------------------------------------------ prolongation
// One thread per fine node (e, i): the physical position of node i of entity
// e (the multilinear image of the Gauss-Lobatto reference node on level 0,
// the node of the child's box above) and the coarse tensor basis of the
// parent's box there; writes row i of P_e (B contiguous values).
template <int D, int Q>
__global__ __launch_bounds__(kSW) void k_prolong_blocks(int64_t n, int level0, const int64_t* __restrict__ cells,
                                                      const double* __restrict__ xyz,
                                                      const double* __restrict__ lo_l,
                                                      const double* __restrict__ hi_l,
                                                      const int64_t* __restrict__ parent,
                                                      const double* __restrict__ lo_c,
                                                      const double* __restrict__ hi_c,
                                                      const double* __restrict__ nodes,
                                                      double* __restrict__ P) {
    constexpr int B = D == 2 ? Q * Q : Q * Q * Q;
    constexpr int NC = 1 << D;
    const int64_t r = (int64_t)blockIdx.x * kSW + threadIdx.x;
    if (r >= n * B) return;
    const int64_t e = r / B;
    const int i = (int)(r - e * B);
    double xi[D], x[D];
    {
        int t = i;
        for (int k = 0; k < D; ++k) {
            xi[k] = nodes[t % Q];
            t /= Q;
        }
    }
    if (level0) {
        for (int a = 0; a < D; ++a) x[a] = 0.0;
        for (int c = 0; c < NC; ++c) {
            double psi = 1.0;
            for (int k = 0; k < D; ++k) psi *= ((c >> k) & 1) ? xi[k] : 1.0 - xi[k];
            const int64_t v = cells[e * NC + c];
            for (int a = 0; a < D; ++a) x[a] += xyz[v * D + a] * psi;
        }
    } else {
        for (int k = 0; k < D; ++k) x[k] = lo_l[e * D + k] + xi[k] * (hi_l[e * D + k] - lo_l[e * D + k]);
    }
    const int64_t K = parent[e];
    double l1[D][Q];
    for (int k = 0; k < D; ++k) {
        const double a = lo_c[K * D + k], w = hi_c[K * D + k] - a;
        const double t = (x[k] - a) / w;
        for (int j = 0; j < Q; ++j) {
            double v = 1.0;
            for (int m = 0; m < Q; ++m)
                if (m != j) v *= (t - nodes[m]) / (nodes[j] - nodes[m]);
            l1[k][j] = v;
        }
    }
    double* out = P + r * B;
    for (int j = 0; j < B; ++j) {
        double v = 1.0;
        int rj = j;
        for (int k = 0; k < D; ++k) {
            v *= l1[k][rj % Q];
            rj /= Q;
        }
        out[j] = v;
    }
}

// ---------------------------------------------------------------- Galerkin
// One workgroup per coarse block (coarse cells first, then coarse faces).
// For every contribution in list order: stage the fine block X and the two
// prolongation blocks in LDS, Y = X P_c (held in registers, then written over
// X), T = P_a^T Y, and accumulate T, T^T or T + T^T into the thread's entries
// of the coarse block.  The order of every sum is fixed, so the result is
// deterministic.
template <int B, int NT>
__global__ __launch_bounds__(NT) void k_galerkin(const double* __restrict__ Ad, const double* __restrict__ Af,
                                                 const int64_t* __restrict__ fc,
                                                 const double* __restrict__ P,
                                                 const int64_t* __restrict__ ptr,
                                                 const int64_t* __restrict__ item, int64_t nC,
                                                 double* __restrict__ outd, double* __restrict__ outf) {
    constexpr int BB = B * B, E = (BB + NT - 1) / NT;
    __shared__ double sX[BB], sPa[BB], sPc[BB];
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x;
    double acc[E];
#pragma unroll
    for (int u = 0; u < E; ++u) acc[u] = 0.0;
    const int64_t i0 = ptr[t], i1 = ptr[t + 1];
    for (int64_t it = i0; it < i1; ++it) {
        const int64_t code = item[it];
        const int mode = (int)(code & 3);
        const int64_t src = code >> 2;
        const double* X = (mode == 0 ? Ad : Af) + src * BB;
        const int64_t ea = mode == 0 ? src : fc[2 * src];
        const int64_t ec = mode == 0 ? src : fc[2 * src + 1];
        for (int k = tid; k < BB; k += NT) {
            sX[k] = X[k];
            sPc[k] = P[ec * BB + k];
            sPa[k] = P[ea * BB + k];
        }
        __syncthreads();
        double y[E];
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int k = tid + u * NT;
            double s = 0.0;
            if (k < BB) {
                const int i = k / B, j = k - (k / B) * B;
#pragma unroll 9
                for (int m = 0; m < B; ++m) s += sX[i * B + m] * sPc[m * B + j];
            }
            y[u] = s;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int k = tid + u * NT;
            if (k < BB) sX[k] = y[u];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int k = tid + u * NT;
            if (k < BB) {
                const int i = k / B, j = k - (k / B) * B;
                double tij = 0.0, tji = 0.0;
                if (mode != 2) {
#pragma unroll 9
                    for (int m = 0; m < B; ++m) tij += sPa[m * B + i] * sX[m * B + j];
                }
                if (mode >= 2) {
#pragma unroll 9
                    for (int m = 0; m < B; ++m) tji += sPa[m * B + j] * sX[m * B + i];
                }
                acc[u] += mode == 3 ? tij + tji : (mode == 2 ? tji : tij);
            }
        }
        __syncthreads();
    }
    double* out = t < nC ? outd + t * BB : outf + (t - nC) * BB;
#pragma unroll
    for (int u = 0; u < E; ++u) {
        const int k = tid + u * NT;
        if (k < BB) out[k] = acc[u];
    }
}

// ----------------------------------------------------------------- Lanczos
// Deterministic workgroup sum (wave shuffles, then the waves in order);
// the result is valid in thread 0.
__device__ double wg_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __shared__ double red[kSW / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kSW / 64; ++w) t += red[w];
    return t;
}

// w = S A S v - beta vp (S = D^-1/2) with the raw blocks and per-cell face
// lists; part[block] = partial (w, v).
template <int B>
__global__ __launch_bounds__(kSW) void k_lz_apply(int64_t n, const double* __restrict__ Ad,
                                                const double* __restrict__ Af,
                                                const int64_t* __restrict__ fc,
                                                const int64_t* __restrict__ cptr,
                                                const int64_t* __restrict__ code,
                                                const double* __restrict__ s,
                                                const double* __restrict__ v,
                                                const double* __restrict__ vp, double beta,
                                                double* __restrict__ w, double* __restrict__ part) {
    constexpr int BB = B * B;
    const int64_t r = (int64_t)blockIdx.x * kSW + threadIdx.x;
    double dv = 0.0;
    if (r < n * B) {
        const int64_t K = r / B;
        const int i = (int)(r - K * B);
        double y = 0.0;
        const double* Dk = Ad + K * BB + i * B;
        for (int j = 0; j < B; ++j) y += Dk[j] * (s[K * B + j] * v[K * B + j]);
        for (int64_t e = cptr[K]; e < cptr[K + 1]; ++e) {
            const int64_t f = code[e] >> 1;
            const bool minus = (code[e] & 1) != 0;
            const int64_t nb = minus ? fc[2 * f] : fc[2 * f + 1];
            const double* F = Af + f * BB;
            double fs = 0.0;
            if (!minus)
                for (int j = 0; j < B; ++j) fs += F[i * B + j] * (s[nb * B + j] * v[nb * B + j]);
            else
                for (int j = 0; j < B; ++j) fs += F[j * B + i] * (s[nb * B + j] * v[nb * B + j]);
            y += fs;
        }
        const double wr = s[r] * y - beta * vp[r];
        w[r] = wr;
        dv = wr * v[r];
    }
    const double t = wg_sum(dv);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// w -= a v with a = sc[0]; part[block] = partial (w, w)
__global__ __launch_bounds__(kSW) void k_lz_orth(int64_t m, const double* __restrict__ sc,
                                               const double* __restrict__ v, double* __restrict__ w,
                                               double* __restrict__ part) {
    const int64_t r = (int64_t)blockIdx.x * kSW + threadIdx.x;
    double q = 0.0;
    if (r < m) {
        const double x = w[r] - sc[0] * v[r];
        w[r] = x;
        q = x * x;
    }
    const double t = wg_sum(q);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out[0] = sum of m partials (one workgroup, fixed order)
__global__ __launch_bounds__(kSW) void k_lz_sum(int64_t m, const double* __restrict__ part,
                                              double* __restrict__ out) {
    double t = 0.0;
    for (int64_t k = threadIdx.x; k < m; k += kSW) t += part[k];
    t = wg_sum(t);
    if (threadIdx.x == 0) out[0] = t;
}

// vp = v; v = w / beta
__global__ __launch_bounds__(kSW) void k_lz_next(int64_t m, double beta, double* __restrict__ v,
                                               double* __restrict__ vp, const double* __restrict__ w) {
    const int64_t r = (int64_t)blockIdx.x * kSW + threadIdx.x;
    if (r < m) {
        vp[r] = v[r];
        v[r] = w[r] / beta;
    }
}

// ------------------------------------------------------------ fine assembly
// (section 3: the SIPDG form a_h with the Gauss-Legendre rules of each cell
// and face, multilinear geometry, per-cell conductivities; the mass term of
// eq. fully_discrete)

// Jacobian J[a][k] = dx_a/dxi_k of the multilinear map at xi, its
// determinant and the inverse transpose.
template <int D>
__device__ void dev_cell_map(const double* X, const double* xi, double* J, double* det, double* JinvT) {
    constexpr int NC = 1 << D;
    for (int a = 0; a < D * D; ++a) J[a] = 0.0;
    for (int c = 0; c < NC; ++c) {
        double f[D], df[D];
        for (int k = 0; k < D; ++k) {
            const int bit = (c >> k) & 1;
            f[k] = bit ? xi[k] : 1.0 - xi[k];
            df[k] = bit ? 1.0 : -1.0;
        }
        for (int k = 0; k < D; ++k) {
            double g = df[k];
            for (int m = 0; m < D; ++m)
                if (m != k) g *= f[m];
            for (int a = 0; a < D; ++a) J[a * D + k] += X[c * D + a] * g;
        }
    }
    if constexpr (D == 2) {
        const double dt = J[0] * J[3] - J[1] * J[2];
        *det = dt;
        JinvT[0] = J[3] / dt;
        JinvT[1] = -J[2] / dt;
        JinvT[2] = -J[1] / dt;
        JinvT[3] = J[0] / dt;
    } else {
        const double *r0 = J, *r1 = J + 3, *r2 = J + 6;
        const double c00 = r1[1] * r2[2] - r1[2] * r2[1];
        const double c01 = r1[2] * r2[0] - r1[0] * r2[2];
        const double c02 = r1[0] * r2[1] - r1[1] * r2[0];
        const double c10 = r0[2] * r2[1] - r0[1] * r2[2];
        const double c11 = r0[0] * r2[2] - r0[2] * r2[0];
        const double c12 = r0[1] * r2[0] - r0[0] * r2[1];
        const double c20 = r0[1] * r1[2] - r0[2] * r1[1];
        const double c21 = r0[2] * r1[0] - r0[0] * r1[2];
        const double c22 = r0[0] * r1[1] - r0[1] * r1[0];
        const double dt = r0[0] * c00 + r0[1] * c01 + r0[2] * c02;
        *det = dt;
        JinvT[0] = c00 / dt; JinvT[1] = c01 / dt; JinvT[2] = c02 / dt;
        JinvT[3] = c10 / dt; JinvT[4] = c11 / dt; JinvT[5] = c12 / dt;
        JinvT[6] = c20 / dt; JinvT[7] = c21 / dt; JinvT[8] = c22 / dt;
    }
}

template <int D>
__device__ void dev_corners(const int64_t* cells, const double* xyz, int64_t c, double* X) {
    constexpr int NC = 1 << D;
    for (int k = 0; k < NC; ++k) {
        const int64_t v = cells[c * NC + k];
        for (int a = 0; a < D; ++a) X[k * D + a] = xyz[v * D + a];
    }
}

// s * (packed symmetric D) -> full D x D
template <int D>
__device__ void dev_unpack_D(const double* Dp, double s, double* Dm) {
    if constexpr (D == 2) {
        Dm[0] = s * Dp[0]; Dm[1] = s * Dp[1];
        Dm[2] = s * Dp[1]; Dm[3] = s * Dp[2];
    } else {
        Dm[0] = s * Dp[0]; Dm[1] = s * Dp[1]; Dm[2] = s * Dp[2];
        Dm[3] = s * Dp[1]; Dm[4] = s * Dp[3]; Dm[5] = s * Dp[4];
        Dm[6] = s * Dp[2]; Dm[7] = s * Dp[4]; Dm[8] = s * Dp[5];
    }
}

// Per cell: w_q |det J| and J^-T at every cell quadrature point (cgeo, 1 + D^2
// values per point), the cell volume and a flag for a non-positive Jacobian.
template <int D>
__global__ __launch_bounds__(kSW) void k_asm_cell_geo(int64_t n, int qc, const int64_t* __restrict__ cells,
                                                    const double* __restrict__ xyz,
                                                    const double* __restrict__ cq_xi,
                                                    const double* __restrict__ cq_w,
                                                    double* __restrict__ cgeo, double* __restrict__ vol,
                                                    int32_t* __restrict__ bad) {
    constexpr int G = 1 + D * D;
    const int64_t c = (int64_t)blockIdx.x * kSW + threadIdx.x;
    if (c >= n) return;
    double X[(1 << D) * D], J[D * D], JiT[D * D], det;
    dev_corners<D>(cells, xyz, c, X);
    double v = 0.0;
    int nb = 0;
    for (int q = 0; q < qc; ++q) {
        dev_cell_map<D>(X, cq_xi + q * D, J, &det, JiT);
        if (!(det > 0.0)) ++nb;
        const double wd = cq_w[q] * fabs(det);
        v += wd;
        double* g = cgeo + (c * qc + q) * G;
        g[0] = wd;
        for (int k = 0; k < D * D; ++k) g[1 + k] = JiT[k];
    }
    vol[c] = v;
    bad[c] = nb;
}

// Per face and face point: dS, sigma, D+ n, D- n, J+^-T, J-^-T (fgeo,
// FG = 2 + 2D + 2D^2 values per point).  n is the unit normal out of the
// plus cell from its geometry; sigma = eta_F mean(n.D+ n, n.D- n) with the
// paper's eta_F = c p(p+1) mean(|F|/|K+|, |F|/|K-|) or a fixed eta.
template <int D>
__global__ __launch_bounds__(kSW) void k_asm_face_geo(
    int64_t nf, int qf, const int64_t* __restrict__ plus, const int64_t* __restrict__ minus,
    const int32_t* __restrict__ axis, const int64_t* __restrict__ cells, const double* __restrict__ xyz,
    const double* __restrict__ Dcell, const double* __restrict__ scale, const double* __restrict__ vol,
    const double* __restrict__ fxi_p, const double* __restrict__ fxi_m, const double* __restrict__ fw,
    int pen_fixed, double eta_in, int p, double* __restrict__ fgeo) {
    constexpr int NP = D * (D + 1) / 2, FG = 2 + 2 * D + 2 * D * D;
    const int64_t f = (int64_t)blockIdx.x * kSW + threadIdx.x;
    if (f >= nf) return;
    const int64_t cp = plus[f], cm = minus[f];
    const int ax = axis[f];
    double Xp[(1 << D) * D], Xm[(1 << D) * D], J[D * D], JiTp[D * D], JiTm[D * D], detp, detm;
    dev_corners<D>(cells, xyz, cp, Xp);
    dev_corners<D>(cells, xyz, cm, Xm);
    double Dp[D * D], Dm[D * D];
    dev_unpack_D<D>(Dcell + cp * NP, scale ? scale[cp] : 1.0, Dp);
    dev_unpack_D<D>(Dcell + cm * NP, scale ? scale[cm] : 1.0, Dm);
    double area = 0.0;
    for (int q = 0; q < qf; ++q) {
        const int o = ax * qf + q;
        dev_cell_map<D>(Xp, fxi_p + o * D, J, &detp, JiTp);
        double nn = 0.0;
        for (int a = 0; a < D; ++a) nn += JiTp[a * D + ax] * JiTp[a * D + ax];
        nn = sqrt(nn);
        area += fw[o] * fabs(detp) * nn;
    }
    const double cpen = eta_in > 0.0 ? eta_in : 1.0;
    const double eta = pen_fixed ? eta_in : cpen * p * (p + 1) * 0.5 * (area / vol[cp] + area / vol[cm]);
    for (int q = 0; q < qf; ++q) {
        const int o = ax * qf + q;
        dev_cell_map<D>(Xp, fxi_p + o * D, J, &detp, JiTp);
        dev_cell_map<D>(Xm, fxi_m + o * D, J, &detm, JiTm);
        double nv[D], nn = 0.0;
        for (int a = 0; a < D; ++a) {
            nv[a] = JiTp[a * D + ax];
            nn += nv[a] * nv[a];
        }
        nn = sqrt(nn);
        for (int a = 0; a < D; ++a) nv[a] /= nn;
        double* g = fgeo + (f * qf + q) * FG;
        g[0] = fw[o] * fabs(detp) * nn;
        double nDn = 0.0;
        for (int a = 0; a < D; ++a) {
            double sp = 0.0, sm = 0.0;
            for (int k = 0; k < D; ++k) {
                sp += Dp[a * D + k] * nv[k];
                sm += Dm[a * D + k] * nv[k];
            }
            g[2 + a] = sp;
            g[2 + D + a] = sm;
        }
        for (int a = 0; a < D; ++a) nDn += 0.5 * nv[a] * (g[2 + a] + g[2 + D + a]);
        g[1] = eta * nDn;
        for (int k = 0; k < D * D; ++k) {
            g[2 + 2 * D + k] = JiTp[k];
            g[2 + 2 * D + D * D + k] = JiTm[k];
        }
    }
}

// conormal flux of basis function i at a face point: (J^-T grad phi_i) . (D n)
template <int D>
__device__ __forceinline__ double face_flux(const double* JiT, const double* gref, const double* Dn) {
    double fl = 0.0;
    for (int a = 0; a < D; ++a) {
        double G = 0.0;
        for (int k = 0; k < D; ++k) G += JiT[a * D + k] * gref[k];
        fl += G * Dn[a];
    }
    return fl;
}

// One thread per cell-block entry (c, i, j): the mass and stiffness
// integrals over the cell, diag = s_K S + cM M, then the same-side face
// terms of every face of the cell in ascending face order.
template <int D, int B>
__global__ __launch_bounds__(kSW) void k_asm_diag(
    int64_t n, const double* __restrict__ cgeo, const double* __restrict__ cq_phi,
    const double* __restrict__ cq_dphi, const double* __restrict__ Dcell, const double* __restrict__ scale,
    double cM, const int64_t* __restrict__ cptr, const int64_t* __restrict__ code,
    const int32_t* __restrict__ axis, int qf, const double* __restrict__ fgeo,
    const double* __restrict__ fphi_p, const double* __restrict__ fphi_m, const double* __restrict__ fg_p,
    const double* __restrict__ fg_m, double* __restrict__ diag, double* __restrict__ mass) {
    constexpr int NP = D * (D + 1) / 2, G = 1 + D * D, FG = 2 + 2 * D + 2 * D * D, BB = B * B;
    const int64_t r = (int64_t)blockIdx.x * kSW + threadIdx.x;
    if (r >= n * BB) return;
    const int64_t c = r / BB;
    const int ij = (int)(r - c * BB), i = ij / B, j = ij - (ij / B) * B;
    double Dc[D * D];
    dev_unpack_D<D>(Dcell + c * NP, 1.0, Dc);
    double Md = 0.0, Sun = 0.0;
    for (int q = 0; q < B; ++q) {   // B = number of cell quadrature points
        const double* g = cgeo + (c * B + q) * G;
        const double wd = g[0];
        const double* JiT = g + 1;
        double Gi[D], Gj[D], DGj[D];
        for (int a = 0; a < D; ++a) {
            double si = 0.0, sj = 0.0;
            for (int k = 0; k < D; ++k) {
                si += JiT[a * D + k] * cq_dphi[(q * B + i) * D + k];
                sj += JiT[a * D + k] * cq_dphi[(q * B + j) * D + k];
            }
            Gi[a] = si;
            Gj[a] = sj;
        }
        for (int a = 0; a < D; ++a) {
            double s = 0.0;
            for (int k = 0; k < D; ++k) s += Dc[a * D + k] * Gj[k];
            DGj[a] = s;
        }
        double s = 0.0;
        for (int a = 0; a < D; ++a) s += Gi[a] * DGj[a];
        Md += wd * cq_phi[q * B + i] * cq_phi[q * B + j];
        Sun += wd * s;
    }
    double v = (scale ? scale[c] : 1.0) * Sun + cM * Md;
    mass[r] = Md;
    for (int64_t e = cptr[c]; e < cptr[c + 1]; ++e) {
        const int64_t f = code[e] >> 1;
        const bool mi = (code[e] & 1) != 0;
        const int ax = axis[f];
        const double* phi = mi ? fphi_m : fphi_p;
        const double* gr = mi ? fg_m : fg_p;
        const double sgn = mi ? -1.0 : 1.0;
        double L = 0.0;
        for (int q = 0; q < qf; ++q) {
            const int o = ax * qf + q;
            const double* g = fgeo + (f * qf + q) * FG;
            const double* Dn = g + 2 + (mi ? D : 0);
            const double* JiT = g + 2 + 2 * D + (mi ? D * D : 0);
            const double ji = sgn * phi[o * B + i], jj = sgn * phi[o * B + j];
            const double fi = face_flux<D>(JiT, gr + (o * B + i) * D, Dn);
            const double fj = face_flux<D>(JiT, gr + (o * B + j) * D, Dn);
            L += g[0] * (-0.5 * ji * fj - 0.5 * fi * jj + g[1] * ji * jj);
        }
        v += L;
    }
    diag[r] = v;
}

// One thread per face-block entry (f, i, j): the coupling of plus-side row i
// with minus-side column j.
template <int D, int B>
__global__ __launch_bounds__(kSW) void k_asm_faces(int64_t nf, const int32_t* __restrict__ axis, int qf,
                                                 const double* __restrict__ fgeo,
                                                 const double* __restrict__ fphi_p,
                                                 const double* __restrict__ fphi_m,
                                                 const double* __restrict__ fg_p,
                                                 const double* __restrict__ fg_m, double* __restrict__ fblk) {
    constexpr int FG = 2 + 2 * D + 2 * D * D, BB = B * B;
    const int64_t r = (int64_t)blockIdx.x * kSW + threadIdx.x;
    if (r >= nf * BB) return;
    const int64_t f = r / BB;
    const int ij = (int)(r - f * BB), i = ij / B, j = ij - (ij / B) * B;
    const int ax = axis[f];
    double L = 0.0;
    for (int q = 0; q < qf; ++q) {
        const int o = ax * qf + q;
        const double* g = fgeo + (f * qf + q) * FG;
        const double ji = fphi_p[o * B + i], jj = -fphi_m[o * B + j];
        const double fi = face_flux<D>(g + 2 + 2 * D, fg_p + (o * B + i) * D, g + 2);
        const double fj = face_flux<D>(g + 2 + 2 * D + D * D, fg_m + (o * B + j) * D, g + 2 + D);
        L += g[0] * (-0.5 * ji * fj - 0.5 * fi * jj + g[1] * ji * jj);
    }
    fblk[r] = L;
}

// set-up temporaries come from the solver's device memory provider and are
// released with the set-up object
struct Owned {
    const DeviceMemory& mem;
    std::vector<void*> ptrs;
    explicit Owned(const DeviceMemory& m) : mem(m) {}
    ~Owned() {
        for (void* p : ptrs) mem.release(p);
    }
};
template <typename T>
T* dev_alloc(Owned& owned, size_t count) {
    void* p = owned.mem.alloc(std::max<size_t>(count, 1) * sizeof(T));
    owned.ptrs.push_back(p);
    return (T*)p;
}
template <typename T>
T* dev_upload(Owned& owned, const std::vector<T>& h) {
    T* d = dev_alloc<T>(owned, h.size());
    if (!h.empty()) DSCHK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}
template <typename T>
void dev_download(std::vector<T>& h, const T* d, size_t count) {
    h.resize(count);
    if (count) DSCHK(hipMemcpy(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost));
}

unsigned grid_for(int64_t threads) { return (unsigned)((threads + kSW - 1) / kSW); }

#define DS_DISPATCH_B(bval, ...)                                                       \
    switch (bval) {                                                                    \
        case 4: { constexpr int BV = 4; __VA_ARGS__; } break;                          \
        case 8: { constexpr int BV = 8; __VA_ARGS__; } break;                          \
        case 9: { constexpr int BV = 9; __VA_ARGS__; } break;                          \
        case 16: { constexpr int BV = 16; __VA_ARGS__; } break;                        \
        case 25: { constexpr int BV = 25; __VA_ARGS__; } break;                        \
        case 27: { constexpr int BV = 27; __VA_ARGS__; } break;                        \
        case 64: { constexpr int BV = 64; __VA_ARGS__; } break;                        \
        default: fail(DGMG_EUNSUPPORTED, "unsupported block size");                    \
    }

}  // namespace

struct DeviceSetup::Impl {
    const Hierarchy& h;
    int d = 0, q = 0, b = 0;
    Owned owned;
    int64_t* cells = nullptr;
    double *xyz = nullptr, *nodes = nullptr;
    struct Op {
        double *diag = nullptr, *fblk = nullptr;
        int64_t* fc = nullptr;
    };
    std::vector<Op> ops;
    std::vector<double*> P;
    std::vector<int64_t*> parent;
    Impl(const Hierarchy& hh, const DeviceMemory& mem) : h(hh), owned(mem) {}
};

DeviceSetup::DeviceSetup(const Hierarchy& h, const RefElement& re, const DeviceMemory& mem) : im(nullptr) {
    std::unique_ptr<Impl> m(new Impl(h, mem));   // released (with its buffers) if an upload fails
    m->d = re.d;
    m->q = re.q;
    m->b = re.b;
    m->ops.resize(h.n_levels);
    m->P.assign(h.n_levels, nullptr);
    m->parent.assign(h.n_levels, nullptr);
    m->cells = dev_upload(m->owned, h.cells);
    m->xyz = dev_upload(m->owned, h.xyz);
    m->nodes = dev_upload(m->owned, re.nodes);
    im = m.release();
}

DeviceSetup::~DeviceSetup() { delete im; }

void DeviceSetup::prolongation(int level, const std::vector<double>& lo_l, const std::vector<double>& hi_l,
                               const std::vector<double>& lo_c, const std::vector<double>& hi_c,
                               std::vector<double>& P) {
    Impl& m = *im;
    const int64_t n = m.h.n_ent[level];
    const int b = m.b;
    double* dlo_l = level ? dev_upload(m.owned, lo_l) : nullptr;
    double* dhi_l = level ? dev_upload(m.owned, hi_l) : nullptr;
    double* dlo_c = dev_upload(m.owned, lo_c);
    double* dhi_c = dev_upload(m.owned, hi_c);
    m.parent[level] = dev_upload(m.owned, m.h.parent[level]);
    m.P[level] = dev_alloc<double>(m.owned, (size_t)n * b * b);
    const unsigned g = grid_for(n * b);
    const int l0 = level == 0 ? 1 : 0;
#define DS_PROLONG(D_, Q_)                                                                              \
    k_prolong_blocks<D_, Q_><<<g, kSW>>>(n, l0, m.cells, m.xyz, dlo_l, dhi_l, m.parent[level], dlo_c, \
                                         dhi_c, m.nodes, m.P[level])
    if (m.d == 2) {
        switch (m.q) {
            case 2: DS_PROLONG(2, 2); break;
            case 3: DS_PROLONG(2, 3); break;
            case 4: DS_PROLONG(2, 4); break;
            case 5: DS_PROLONG(2, 5); break;
            default: fail(DGMG_EUNSUPPORTED, "unsupported degree");
        }
    } else {
        switch (m.q) {
            case 2: DS_PROLONG(3, 2); break;
            case 3: DS_PROLONG(3, 3); break;
            case 4: DS_PROLONG(3, 4); break;
            default: fail(DGMG_EUNSUPPORTED, "unsupported degree");
        }
    }
#undef DS_PROLONG
    DSCHK(hipGetLastError());
    dev_download(P, m.P[level], (size_t)n * b * b);
}

void DeviceSetup::assemble_fine(const Faces& F, const RefElement& re, const dgmg_disc& disc,
                                const dgmg_physics& ph, double cM, BlockOp& A0, std::vector<double>& mass) {
    Impl& m = *im;
    const int d = re.d, b = re.b, bb = b * b, np = d * (d + 1) / 2;
    const int64_t n = m.h.n_cells, nf = (int64_t)F.plus.size();
    FaceRef fr;
    fr.init(re);
    const int qf = fr.qf;
    // inputs and reference tables
    std::vector<double> Dh(ph.D_cell, ph.D_cell + (size_t)n * np);
    double* Dcell = dev_upload(m.owned, Dh);
    double* scale = nullptr;
    if (ph.cell_scale) scale = dev_upload(m.owned, std::vector<double>(ph.cell_scale, ph.cell_scale + n));
    double* cq_xi = dev_upload(m.owned, re.cq_xi);
    double* cq_w = dev_upload(m.owned, re.cq_w);
    double* cq_phi = dev_upload(m.owned, re.cq_phi);
    double* cq_dphi = dev_upload(m.owned, re.cq_dphi);
    double* fxi_p = dev_upload(m.owned, fr.xi_p);
    double* fxi_m = dev_upload(m.owned, fr.xi_m);
    double* fw = dev_upload(m.owned, fr.w);
    double* fphi_p = dev_upload(m.owned, fr.phi_p);
    double* fphi_m = dev_upload(m.owned, fr.phi_m);
    double* fg_p = dev_upload(m.owned, fr.g_p);
    double* fg_m = dev_upload(m.owned, fr.g_m);
    int64_t* dplus = dev_upload(m.owned, F.plus);
    int64_t* dminus = dev_upload(m.owned, F.minus);
    std::vector<int32_t> ax32(F.axis.begin(), F.axis.end());
    int32_t* daxis = dev_upload(m.owned, ax32);
    // structure of the fine operator
    A0.n = n;
    A0.b = b;
    A0.nf = nf;
    A0.fc.resize((size_t)nf * 2);
    for (int64_t f = 0; f < nf; ++f) {
        A0.fc[2 * f] = F.plus[f];
        A0.fc[2 * f + 1] = F.minus[f];
    }
    std::vector<int64_t> cptr, code;
    cell_face_lists(A0, cptr, code);
    int64_t* dcptr = dev_upload(m.owned, cptr);
    int64_t* dcode = dev_upload(m.owned, code);
    // geometry
    const int G = 1 + d * d, FG = 2 + 2 * d + 2 * d * d;
    double* cgeo = dev_alloc<double>(m.owned, (size_t)n * re.qc * G);
    double* vol = dev_alloc<double>(m.owned, n);
    int32_t* bad = dev_alloc<int32_t>(m.owned, n);
    double* fgeo = dev_alloc<double>(m.owned, (size_t)nf * qf * FG);
    Impl::Op& op = m.ops[0];
    op.diag = dev_alloc<double>(m.owned, (size_t)n * bb);
    op.fblk = dev_alloc<double>(m.owned, (size_t)nf * bb);
    op.fc = dev_upload(m.owned, A0.fc);
    double* dmass = dev_alloc<double>(m.owned, (size_t)n * bb);
    const int pen_fixed = disc.penalty_mode == DGMG_PENALTY_FIXED ? 1 : 0;
    auto run = [&](auto dtag) {
        constexpr int D = decltype(dtag)::value;
        if (n > 0)
            k_asm_cell_geo<D><<<grid_for(n), kSW>>>(n, re.qc, m.cells, m.xyz, cq_xi, cq_w, cgeo, vol, bad);
        DSCHK(hipGetLastError());
        std::vector<int32_t> hb;
        dev_download(hb, bad, (size_t)n);
        for (int32_t v : hb)
            if (v) fail(DGMG_EINVAL, "non-positive Jacobian determinant in the mesh");
        if (nf > 0)
            k_asm_face_geo<D><<<grid_for(nf), kSW>>>(nf, qf, dplus, dminus, daxis, m.cells, m.xyz, Dcell, scale,
                                                     vol, fxi_p, fxi_m, fw, pen_fixed, disc.eta, re.p, fgeo);
        DSCHK(hipGetLastError());
        DS_DISPATCH_B(b, {
            if constexpr ((D == 2 && (BV == 4 || BV == 9 || BV == 16 || BV == 25)) ||
                          (D == 3 && (BV == 8 || BV == 27 || BV == 64))) {
                if (n > 0)
                    k_asm_diag<D, BV><<<grid_for(n * bb), kSW>>>(n, cgeo, cq_phi, cq_dphi, Dcell, scale, cM,
                                                                  dcptr, dcode, daxis, qf, fgeo, fphi_p, fphi_m,
                                                                  fg_p, fg_m, op.diag, dmass);
                if (nf > 0)
                    k_asm_faces<D, BV><<<grid_for(nf * bb), kSW>>>(nf, daxis, qf, fgeo, fphi_p, fphi_m, fg_p,
                                                                   fg_m, op.fblk);
            } else {
                fail(DGMG_EUNSUPPORTED, "block size does not match the dimension");
            }
        });
        DSCHK(hipGetLastError());
    };
    if (d == 2)
        run(std::integral_constant<int, 2>{});
    else
        run(std::integral_constant<int, 3>{});
    dev_download(A0.diag, op.diag, (size_t)n * bb);
    dev_download(A0.fblk, op.fblk, (size_t)nf * bb);
    dev_download(mass, dmass, (size_t)n * bb);
}

void DeviceSetup::set_fine(const BlockOp& A0) {
    Impl& m = *im;
    if (m.ops[0].diag) return;   // assembled here
    m.ops[0].diag = dev_upload(m.owned, A0.diag);
    m.ops[0].fblk = dev_upload(m.owned, A0.fblk);
    m.ops[0].fc = dev_upload(m.owned, A0.fc);
}

void DeviceSetup::galerkin(int level, const BlockOp& A, BlockOp& Ac) {
    Impl& m = *im;
    if (!m.ops[level].diag || !m.P[level]) fail(DGMG_EINVAL, "device Galerkin product without A_l or P_l");
    const int b = m.b, bb = b * b;
    const int64_t nC = m.h.n_ent[level + 1];
    GalerkinPlan plan;
    galerkin_plan(A, m.h.parent[level], nC, Ac, plan);
    int64_t* dptr = dev_upload(m.owned, plan.ptr);
    int64_t* ditem = dev_upload(m.owned, plan.item);
    Impl::Op& out = m.ops[level + 1];
    out.diag = dev_alloc<double>(m.owned, (size_t)nC * bb);
    out.fblk = dev_alloc<double>(m.owned, (size_t)Ac.nf * bb);
    out.fc = dev_upload(m.owned, Ac.fc);
    const int64_t nt = nC + Ac.nf;
    const Impl::Op& in = m.ops[level];
    if (nt > 0) {
        DS_DISPATCH_B(b, {
            constexpr int NT = BV * BV <= 64 ? 64 : (BV * BV <= 128 ? 128 : 256);
            k_galerkin<BV, NT><<<(unsigned)nt, NT>>>(in.diag, in.fblk, in.fc, m.P[level], dptr, ditem, nC,
                                                     out.diag, out.fblk);
        });
        DSCHK(hipGetLastError());
    }
    dev_download(Ac.diag, out.diag, (size_t)nC * bb);
    dev_download(Ac.fblk, out.fblk, (size_t)Ac.nf * bb);
}

double DeviceSetup::lanczos_theta_max(int level, const BlockOp& A, int steps) {
    Impl& m = *im;
    const Impl::Op& op = m.ops[level];
    if (!op.diag) fail(DGMG_EINVAL, "device Lanczos without A_l");
    const int b = A.b;
    const int64_t n = A.n * b;
    std::vector<double> sh(n), v0;
    for (int64_t K = 0; K < A.n; ++K)
        for (int i = 0; i < b; ++i) sh[K * b + i] = 1.0 / std::sqrt(A.diag[((size_t)K * b + i) * b + i]);
    lanczos_start(n, v0);
    std::vector<int64_t> cptr, code;
    cell_face_lists(A, cptr, code);
    // work vectors are released with the set-up object; a level's vectors
    // are small next to its blocks
    double* s = dev_upload(m.owned, sh);
    double* v = dev_upload(m.owned, v0);
    double* vp = dev_alloc<double>(m.owned, n);
    DSCHK(hipMemset(vp, 0, n * sizeof(double)));
    double* w = dev_alloc<double>(m.owned, n);
    const unsigned g = grid_for(n);
    double* part = dev_alloc<double>(m.owned, g);
    double* sc = dev_alloc<double>(m.owned, 2);
    int64_t* dptr = dev_upload(m.owned, cptr);
    int64_t* dcode = dev_upload(m.owned, code);
    std::vector<double> al, be;
    double beta = 0.0;
    const int64_t mmax = std::min<int64_t>(steps, n);
    for (int64_t j = 0; j < mmax; ++j) {
        DS_DISPATCH_B(b, {
            k_lz_apply<BV><<<g, kSW>>>(A.n, op.diag, op.fblk, op.fc, dptr, dcode, s, v, vp, beta, w, part);
        });
        k_lz_sum<<<1, kSW>>>(g, part, sc);
        k_lz_orth<<<g, kSW>>>(n, sc, v, w, part);
        k_lz_sum<<<1, kSW>>>(g, part, sc + 1);
        DSCHK(hipGetLastError());
        double hs[2];
        DSCHK(hipMemcpy(hs, sc, sizeof(hs), hipMemcpyDeviceToHost));
        al.push_back(hs[0]);
        beta = std::sqrt(hs[1]);
        if (beta < 1e-14 || j == mmax - 1) break;
        be.push_back(beta);
        k_lz_next<<<g, kSW>>>(n, beta, v, vp, w);
    }
    DSCHK(hipGetLastError());
    be.resize(al.size() > 0 ? al.size() - 1 : 0);
    if (al.size() == 1) return al[0];
    return tridiag_max_eig(al, be);
}

}  // namespace dgmg
