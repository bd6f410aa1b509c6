// Pointwise ionic update and load-vector kernels (section 2.2 models,
// section 3.1 time stepping with ionic current interpolation).
//
// Every supported model has gate dynamics affine in each gate at fixed
// potential, dw/dt = c1(u) w + c0(u), so the BDF2 gate update driven by the
// extrapolated potential U* = 2 U_n - U_{n-1} is closed-form:
//   W_{n+1} = (4 W_n - W_{n-1} + 2 dt c0(U*)) / (3 - 2 dt c1(U*)).
// Parameter vectors:
//   FHN [k, a, eps, Gamma]: I = k u (u-a)(u-1) + w,  dw/dt = eps (u - Gamma w)
//   AP  [k, a, eps0]:       I = k u (u-a)(u-1) + u v, dv/dt = eps0 (-v - k u (u-a-1))
//   BO  28 values (tau_o', tau_o'', tau_so', tau_so'', tau_si, tau_fi, tau_1+,
//       tau_1', tau_1'', tau_2', tau_2'', tau_3', tau_3'', tau_2+, tau_2inf,
//       k_2, k_3, k_so, w*_inf, V_1, V_1m, V_2, V_2m, V_3, V_hat, V_o, V_so, u_o)
//       with the Heaviside variants read as: sharp H at V_1m in a_0 and w0_inf,
//       smooth H (k_2) at V_2m in a_1, smooth H (k_3) at V_3 for w2_inf, smooth
//       H (k_so) at V_so in the second so-term; sharp H(0) = 1/2.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgmg {

constexpr int kMaxParams = 32;
struct IonicParams {
    int model, S, bdf;
    double dt, chi, Cm;
    double p[kMaxParams];
};

__device__ __forceinline__ double hs(double z) { return z > 0.0 ? 1.0 : (z < 0.0 ? 0.0 : 0.5); }
__device__ __forceinline__ double hk(double z, double k) { return 0.5 * (1.0 + tanh(k * z)); }

enum BOi {
    TO1, TO2, TSO1, TSO2, TSI, TFI, T1P, T1M1, T1M2, T2M1, T2M2, T3M1, T3M2, T2P, T2INF, K2, K3,
    KSO, WINF, V1, V1M, V2, V2M, V3, VHAT, VO, VSO, UO
};

// gate coefficients c1[s], c0[s] at potential u
__device__ __forceinline__ void gate_coeffs(const IonicParams& P, double u, double* c1, double* c0) {
    const double* p = P.p;
    if (P.model == 0) {
        c1[0] = -p[2] * p[3];
        c0[0] = p[2] * u;
    } else if (P.model == 1) {
        c1[0] = -p[2];
        c0[0] = -p[2] * p[0] * u * (u - p[1] - 1.0);
    } else {
        const double H1 = hs(u - p[V1]), H2 = hs(u - p[V2]), H1m = hs(u - p[V1M]);
        const double H2m = hk(u - p[V2M], p[K2]), Ho = hs(u - p[VO]);
        const double a0 = (1.0 - H1) / (H1m * (p[T1M2] - p[T1M1]) + p[T1M1]);
        const double a1 = (1.0 - H2) / (H2m * (p[T2M2] - p[T2M1]) + p[T2M1]);
        const double a2 = 1.0 / (H2 * (p[T3M2] - p[T3M1]) + p[T3M1]);
        const double b0 = -H1 / p[T1P], b1 = -H2 / p[T2P];
        const double w0i = 1.0 - H1m;
        const double w1i = Ho * (p[WINF] - 1.0 + u / p[T2INF]) + 1.0 - u / p[T2INF];
        const double w2i = hk(u - p[V3], p[K3]);
        c1[0] = b0 - a0; c0[0] = a0 * w0i;
        c1[1] = b1 - a1; c0[1] = a1 * w1i;
        c1[2] = -a2;     c0[2] = a2 * w2i;
    }
}

__device__ __forceinline__ double ionic_current(const IonicParams& P, double u, const double* w) {
    const double* p = P.p;
    if (P.model == 0) return p[0] * u * (u - p[1]) * (u - 1.0) + w[0];
    if (P.model == 1) return p[0] * u * (u - p[1]) * (u - 1.0) + u * w[0];
    const double H1 = hs(u - p[V1]), H2 = hs(u - p[V2]), Ho = hs(u - p[VO]);
    const double Hso = hk(u - p[VSO], p[KSO]);
    const double Ifi = -H1 * (u - p[V1]) * (p[VHAT] - u) * w[0] / p[TFI];
    const double Isi = -H2 * w[1] * w[2] / p[TSI];
    const double Iso = (1.0 - H2) * (u - p[UO]) / (Ho * (p[TO2] - p[TO1]) + p[TO1]) +
                       H2 / (Hso * (p[TSO2] - p[TSO1]) + p[TSO1]);
    return Ifi + Isi + Iso;
}

// W_next (may alias Wprev) and g = I_ion(U*, W_next) at every DoF.
__global__ __launch_bounds__(256) void k_ionic(int64_t N, IonicParams P, const double* __restrict__ U,
                                               const double* __restrict__ Up,
                                               const double* __restrict__ W, const double* Wp,
                                               double* Wn, double* __restrict__ g) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= N) return;
    const double us = P.bdf == 2 ? 2.0 * U[t] - Up[t] : U[t];
    double c1[3], c0[3], w[3];
    gate_coeffs(P, us, c1, c0);
    for (int s = 0; s < P.S; ++s) {
        const double wn = W[s * N + t];
        if (P.bdf == 2)
            w[s] = (4.0 * wn - Wp[s * N + t] + 2.0 * P.dt * c0[s]) / (3.0 - 2.0 * P.dt * c1[s]);
        else
            w[s] = (wn + P.dt * c0[s]) / (1.0 - P.dt * c1[s]);
    }
    for (int s = 0; s < P.S; ++s) Wn[s * N + t] = w[s];
    g[t] = ionic_current(P, us, w);
}

// Load vector of the step, per cell: f = cU * (4 U - Uprev) + iapp - chi g
// (BDF2; backward Euler uses cU * U), b = M_K f.  When xout is set it receives
// U (the warm start), and may alias Uprev: all reads of the cell happen before
// the workgroup barrier.  Workgroups hold whole cells (blockDim = B * cells).
template <int B>
__global__ __launch_bounds__(256) void k_rhs(int32_t n, IonicParams P, double cU,
                                             const double* __restrict__ mass, const double* U,
                                             const double* Up, const double* __restrict__ iapp,
                                             const double* __restrict__ g, double* __restrict__ b,
                                             double* xout) {
    __shared__ double f[256];
    const int cells_per = blockDim.x / B;
    const int lc = threadIdx.x / B, i = threadIdx.x - lc * B;
    const int cell = blockIdx.x * cells_per + lc;
    const bool act = lc < cells_per && cell < n;
    const int64_t t = (int64_t)cell * B + i;
    double u = 0.0;
    if (act) {
        u = U[t];
        const double hist = P.bdf == 2 ? 4.0 * u - Up[t] : u;
        f[threadIdx.x] = cU * hist + (iapp ? iapp[t] : 0.0) - P.chi * g[t];
    }
    __syncthreads();
    if (!act) return;
    // column-major (i, j) at j*B + i, block stride padded to whole 16-byte vectors
    const double* M = mass + (size_t)cell * ((B * B + 1) / 2 * 2) + i;
    const double* fc = f + lc * B;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) acc += M[j * B] * fc[j];
    b[t] = acc;
    if (xout) xout[t] = u;
}

// b = M_K f per cell (no history terms).
template <int B>
__global__ __launch_bounds__(256) void k_mass(int32_t n, const double* __restrict__ mass,
                                              const double* __restrict__ fv, double* __restrict__ b) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int cell = t / B, i = t - cell * B;
    if (cell >= n) return;
    const double* M = mass + (size_t)cell * ((B * B + 1) / 2 * 2) + i;
    const double* fc = fv + (size_t)cell * B;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) acc += M[j * B] * fc[j];
    b[t] = acc;
}

}  // namespace dgmg
