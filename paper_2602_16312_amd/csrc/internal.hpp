// Internal declarations shared by the host setup and the device solver.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dgmg.h"

namespace dgmg {

// Error carrying a DGMG_* code; converted to a return value at the C ABI.
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void set_last_error(const std::string& msg);

// ---------------------------------------------------------------- reference
constexpr int kMaxQ = 5;                      // points per direction, p <= 4
struct RefElement {
    int d = 0, p = 0, q = 0, b = 0;          // q = p + 1 points per direction
    std::vector<double> nodes;                // Gauss-Lobatto nodes on [0,1]
    std::vector<double> gx, gw;               // Gauss-Legendre rule on [0,1], p+1 points
    // cell quadrature (tensor), qc = q^d points
    int qc = 0;
    std::vector<double> cq_xi, cq_w;          // [qc][d], [qc]
    std::vector<double> cq_phi, cq_dphi;      // [qc][b], [qc][b][d]
    void init(int dim, int deg);
};

// Face rule of each axis on the reference cell: for axis a and face point
// iq, the reference points on the upper (xi_a = 1, "plus" side of a face) and
// lower (xi_a = 0, "minus" side) cell faces, the weight, and the basis values
// and reference gradients there ([d][qf][...] arrays).
struct FaceRef {
    int qf = 0;                                   // (p+1)^(d-1) points per face
    std::vector<double> xi_p, xi_m, w;            // [d][qf][d], [d][qf][d], [d][qf]
    std::vector<double> phi_p, phi_m, g_p, g_m;   // [d][qf][b], [d][qf][b][d]
    void init(const RefElement& re);
};

// 1D Lagrange values and derivatives on `nodes` at x.
void lagrange1d(const std::vector<double>& nodes, double x, double* val, double* der);
// tensor basis values (and gradients if grad != nullptr) at reference point xi
void tensor_eval(const RefElement& re, const double* xi, double* phi, double* grad);
// multilinear geometry of a cell with corners X[2^d][d] at xi: x, J[a][k], det, JinvT[a][k]
void cell_map(int d, const double* X, const double* xi, double* x, double* J, double* det,
              double* JinvT);

// ---------------------------------------------------------------- hierarchy
struct Hierarchy {
    int dim = 0;
    int64_t n_vert = 0, n_cells = 0;
    std::vector<double> xyz;                  // n_vert * dim
    std::vector<int64_t> cells;               // n_cells * 2^dim
    int n_levels = 1;
    std::vector<int64_t> n_ent;               // per level
    std::vector<std::vector<int64_t>> parent; // parent[l][e] on level l+1, l < L-1
};

// ---------------------------------------------------------------- operators
// Block-sparse symmetric level operator: one b x b block per cell (row-major),
// one b x b block per face pair (rows of `plus`, columns of `minus`).
struct BlockOp {
    int64_t n = 0, nf = 0;
    int b = 0;
    std::vector<double> diag;                 // n * b * b
    std::vector<int64_t> fc;                  // nf * 2 (plus, minus)
    std::vector<double> fblk;                 // nf * b * b
};

struct Faces {                                 // interior faces of the fine mesh
    std::vector<int64_t> plus, minus;
    std::vector<int> axis;
};

Faces find_faces(const Hierarchy& h);
// dA/ds_K pieces: unscaled cell stiffness S_K (n x b x b, row-major) and, per
// face, the face matrices of each side alone (2 x 2b x 2b over [K+, K-] DoFs)
struct AdjointBlocks {
    std::vector<double> S, X;
};
// Assembles A_0 = cM * M + A (cell and face blocks) and the per-cell mass blocks.
void assemble_fine(const Hierarchy& h, const Faces& F, const RefElement& re,
                   const dgmg_disc& disc, const dgmg_physics& ph, double cM, BlockOp& A0,
                   std::vector<double>& mass, AdjointBlocks* adj = nullptr);

// Prolongation blocks P_e (n_l x b x b, row-major: fine node i, coarse basis j)
// from level l+1 to level l, with per-level bounding boxes.
void prolongation_blocks(const Hierarchy& h, const RefElement& re, int level,
                         const std::vector<double>& lo_l, const std::vector<double>& hi_l,
                         const std::vector<double>& lo_c, const std::vector<double>& hi_c,
                         std::vector<double>& P);
void level_boxes(const Hierarchy& h, int level, std::vector<double>& lo, std::vector<double>& hi);
// Integer structure of A_{l+1} = P^T A_l P: the coarse face list (plus =
// smaller coarse id) and, per coarse entity t (cells 0..n_coarse-1, then
// faces), the fine contributions item[ptr[t]..ptr[t+1]) in summation order,
// each (source << 2) | mode: mode 0 = P_e^T A_ee P_e of fine cell e = source;
// for fine face f = source with T = P_{e+}^T A_f P_{e-}: 1 = T, 2 = T^T,
// 3 = T + T^T (a face between two children of one agglomerate).
struct GalerkinPlan {
    std::vector<int64_t> ptr, item;
};
void galerkin_plan(const BlockOp& A, const std::vector<int64_t>& parent, int64_t n_coarse,
                   BlockOp& Ac, GalerkinPlan& plan);
void galerkin(const BlockOp& A, const std::vector<double>& P, const std::vector<int64_t>& parent,
              int64_t n_coarse, BlockOp& Ac);
void host_apply(const BlockOp& A, const double* x, double* y);
// per-cell face lists: faces of cell K are code[ptr[K]..ptr[K+1]),
// code = face << 1 | (K is the minus side)
void cell_face_lists(const BlockOp& A, std::vector<int64_t>& ptr, std::vector<int64_t>& code);
double lanczos_theta_max(const BlockOp& A, int steps, const std::vector<double>* chol = nullptr);
void cell_block_factors(const BlockOp& A, std::vector<double>& Lc, std::vector<double>& Dinv);
// Largest eigenvalue of the symmetric tridiagonal matrix (a, off-diagonal bt).
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& bt);
// Lanczos start vector: v_i = frac((i+1) * golden ratio conjugate) - 1/2, normalised
void lanczos_start(int64_t n, std::vector<double>& v);

// Device memory of the library's own buffers: the caller's allocator when one
// was given at set-up, hipMalloc / hipFree otherwise.
struct DeviceMemory {
    dgmg_allocator user{};
    bool has_user = false;
    void* alloc(size_t bytes) const;    // fails with DGMG_ENOMEM
    void release(void* p) const noexcept;
};

// Device set-up (prolongation blocks, Galerkin products and Lanczos
// estimates on the GPU); holds its device buffers until destroyed.
class DeviceSetup {
  public:
    DeviceSetup(const Hierarchy& h, const RefElement& re, const DeviceMemory& mem);
    ~DeviceSetup();
    DeviceSetup(const DeviceSetup&) = delete;
    DeviceSetup& operator=(const DeviceSetup&) = delete;
    // P_l (level l -> l+1 blocks) on the device; host copy into P
    void prolongation(int level, const std::vector<double>& lo_l, const std::vector<double>& hi_l,
                      const std::vector<double>& lo_c, const std::vector<double>& hi_c,
                      std::vector<double>& P);
    // uploads the fine operator A_0 (unless it was assembled on the device)
    void set_fine(const BlockOp& A0);
    // A_0 = cM M + A and the mass blocks assembled on the device (the blocks
    // stay there for the Galerkin products); host copies into A0 and mass.
    void assemble_fine(const Faces& F, const RefElement& re, const dgmg_disc& disc,
                       const dgmg_physics& ph, double cM, BlockOp& A0, std::vector<double>& mass);
    // A_{l+1} = P_l^T A_l P_l on the device (needs A_l and P_l there); host copy into Ac
    void galerkin(int level, const BlockOp& A, BlockOp& Ac);
    // largest Ritz value of `steps` Lanczos steps on D^-1/2 A_l D^-1/2 (device A_l)
    double lanczos_theta_max(int level, const BlockOp& A, int steps);

  private:
    struct Impl;
    Impl* im;
};
// dense coarse operator, in-place lower Cholesky and explicit inverse
void dense_from_blocks(const BlockOp& A, std::vector<double>& dense);
void cholesky_inverse(std::vector<double>& a, int64_t n);

}  // namespace dgmg
