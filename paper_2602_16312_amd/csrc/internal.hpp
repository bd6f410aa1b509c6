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
void galerkin(const BlockOp& A, const std::vector<double>& P, const std::vector<int64_t>& parent,
              int64_t n_coarse, BlockOp& Ac);
void host_apply(const BlockOp& A, const double* x, double* y);
double lanczos_theta_max(const BlockOp& A, int steps);
// dense coarse operator, in-place lower Cholesky and explicit inverse
void dense_from_blocks(const BlockOp& A, std::vector<double>& dense);
void cholesky_inverse(std::vector<double>& a, int64_t n);

}  // namespace dgmg
