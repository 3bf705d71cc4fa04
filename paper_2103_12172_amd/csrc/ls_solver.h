// Device least-squares solve of the reduced interface system.
#pragma once

#include <vector>

#include "ap_solver.h"

namespace mdp {

struct LSResult {
    double rel_residual = 0.0;  // ||A x - F|| / ||F||
    double cond = 0.0;          // estimate of cond_2 of the column-equilibrated A (0 if not requested)
    bool shifted = false;       // the shifted first pass was needed
    int passes = 0;
    double flops = 0.0;         // algorithmic flops of the method's steps (semi-normal path)
};

// Host description of the block-sparse interface matrix: subdomain i's rows
// form the dense block A_i (m_i x s_i); packed column pc is coefA Q_i(:, colA)
// + coefB Q_i(:, colB) and column pc_gcol[pc] of Qbar.
// Steps of the blocked Cholesky: each step lists the widths (1..64) of its
// mutually uncoupled diagonal sub-blocks, in column order.
using CholPlan = std::vector<std::vector<int>>;
CholPlan chol_plan_uniform(int nc);   // one 64-column block per step

// Elimination tree of the multifrontal Cholesky: subdomains split in halves
// along the longer extent of their centres, down to one subdomain per leaf; a
// column is eliminated at the lowest node whose subdomains hold every subdomain
// that touches it (nested dissection: a node eliminates the interfaces between
// its two halves).
struct MFHost {
    struct Node {
        int e = 0, b = 0, sub = -1, kid[2] = {-1, -1}, height = 0;
        std::vector<int> idx;      // front position -> global column (eliminated first, then boundary)
        std::vector<int> kpos[2];  // child's boundary position -> front position
        std::vector<int> inv[2];   // front position -> child's boundary position, or -1
        std::vector<int> spos;     // leaf: front position -> column of its subdomain's Gram block
        size_t G = 0, L = 0, Z = 0, W = 0, z = 0, cw = 0;   // arena offsets (complex entries)
    };
    // one batched Cholesky step: 64-column panel s of every front of one height with e > 64 s
    struct Step {
        int height, entry0, count, max_roles;   // max_roles: slab workgroups of one entry
        int max_tiles64, max_tiles32;           // update workgroups of one entry (64 x 64, 32 x 32 tiles)
        long tiles64;                           // 64 x 64 update tiles of all entries
        double diag_flops, panel_flops, update_flops, diag_bytes, panel_bytes, update_bytes;
    };
    std::vector<Node> nodes;
    std::vector<std::vector<int>> by_height;   // nodes of each height (leaves: 0)
    std::vector<size_t> lzw;                   // per height: arena range [lzw[h], lzw[h+1]) of its L, Z, W
    std::vector<int> h_max_e, h_max_b;         // per height: largest eliminated and boundary counts
    std::vector<Step> steps;                   // heights in order, panels in order within a height
    std::vector<int> entry_node;               // node of every step entry
    std::vector<int> entry_kb;                 // first column of every step entry's panel
    int max_f = 0, max_e = 0, lds_fwd = 0, lds_bwd = 0;   // largest front, e; LDS entries of the substitutions
    size_t arena = 0;                          // complex entries of the factor arena
    double flops = 0.0;                        // partial factorisations (complex, 8 per multiply-add)
};

struct PackedHost {
    int n_sub = 0, nc = 0, total_pc = 0, max_m = 0, max_s = 0;
    std::vector<double> cx, cy;   // subdomain centres (elimination tree of the multifrontal route)
    bool multifrontal = false;
    MFHost mf;
    CholPlan steps;   // empty: one 64-column block per step
    std::vector<const double2*> Q;
    std::vector<int> m, s, pc_sub, pc_p, pc_gcol, pc_start;
    std::vector<long> off, roff;
    std::vector<int4> pc_cols;
    std::vector<double2> pc_coef;
};

// Blocked Cholesky G + shift I = L L^* and Linv = L^{-1} of an order-nc Hermitian
// positive definite G (lower triangle read and overwritten, ld nc, device);
// L and Linv (nc x nc, ld nc) get zero upper triangles; W is nc x nc scratch;
// a breakdown sets *info_dev (first failing pivot, 1-based) if it is zero.
// Per-launch timing goes to *pr when it is set and enabled.
// The steps follow `plan` (default: one 64-column block per step); sub-blocks of
// one step must not couple (G vanishes between them).
// Returns the algorithmic flops of the factorisation and inverse as computed (dense blocks).
double cholesky_and_inverse(double2* G, double2* L, double2* Linv, double2* W, int* info_dev, int nc, double shift,
                            hipStream_t st, Profiler* pr = nullptr, const CholPlan* plan = nullptr);

// Device tables of the packed solve: offsets into a caller's upload image.
struct PackedTables {
    size_t Q, m, s, off, roff, sub, p, gcol, start, cols, coef, zb;
    size_t gc_start, gc_list;   // global column -> its packed columns (CSR)
    int nsplit;
    size_t mf_nodes, mf_lists, mf_steps;  // multifrontal: node table, node lists by height, step entries
    std::vector<size_t> mf_list_off;      // start of each height's list (entries)
};

// Symbolic phase of the multifrontal route (h.pc_* and h.cx, h.cy set).
MFHost mf_plan(const PackedHost& h);

// Grow the workspaces for h and append the packed solve's tables to blob.
PackedTables ls_packed_tables(Workspace& ws, const PackedHost& h, HostBlob& blob);

// Corrected semi-normal equations on the packed matrix; F is the stacked
// right-hand side (device), `image` the device copy of the blob that holds the
// tables t.  x_out (device) receives the solution.  Synchronises the stream
// once in the common case (convergence check and residual norms together).
// Sets *fallback (and returns) when the Cholesky of the Gram matrix breaks
// down or the refinement does not contract.
// reuse: the workspaces still hold the equilibrated packed matrix and the Gram factor of the
// same system (only F differs from the call that built them): assembly and factorisation are skipped.
LSResult ls_solve_packed(Workspace& ws, const PackedHost& h, const char* image, const PackedTables& t,
                         const double2* F, double2* x_out, bool want_cond, hipStream_t st, bool* fallback,
                         bool reuse = false);

// G^{-1} v with the Gram factor left by the last ls_solve_packed on ws (same h, image and
// tables; G the Gram matrix of the column-equilibrated packed matrix); out must not alias v.
void ls_packed_factor_solve(Workspace& ws, const PackedHost& h, const char* image, const PackedTables& tb,
                            const double2* v, double2* out, hipStream_t st);

// min ||A x - F||_2 for A (m x nc, column-major, ld m, device; overwritten) and
// F (m, device); x_out (nc, device).
LSResult ls_solve(Workspace& ws, double2* A, const double2* F, int m, int nc, double2* x_out, bool want_cond,
                  hipStream_t st);

}  // namespace mdp
