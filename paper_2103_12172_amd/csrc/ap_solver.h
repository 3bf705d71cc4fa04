// Batched auxiliary-problem solver (host orchestration).
#pragma once

#include <functional>

#include "mdp_internal.h"

namespace mdp {

StencilCoef stencil_coef(double h, double k);
EndRowCoef end_row_coef(double h, double k);

// Device constants of one (n, h, k) auxiliary problem.
struct APPlan {
    int n;
    double h, k;
    Fold f;
    StencilCoef sc;
    EndRowCoef ec;
    double min_pivot_ratio;  // smallest |pivot| / row scale over all modes (host check)
    DevBuf Sf64, Si64, Sf32, Si32;     // block-diagonal sine matrices (W x W)
    DevBuf fac64, fac32, colc64, colc32;  // tridiagonal LU factors per mode
    DevBuf lf64, rf64;    // the same l_m and r_m as interleaved complex [(n+1)][W] (fused projector sweep)
    APPlan(int n, double h, double k);
};

// Least-squares buffers (grow-only).
struct LSWork {
    DevBuf G, L, Linv[3], T, A0, Aq, vec, norms, flags;
};

// Packed interface matrix buffers (grow-only).
struct PackedWork {
    DevBuf dQ, dm, ds, doff, droff, dsub, dp, dgcol, dstart, dcols, dcoef, Ap, Gi, dzb;
};

// Interface assembly and reconstruction buffers (grow-only).
struct CallWork {
    DevBuf qsrc, qld, roff, cmap, coef, kcol, kval, koff, F, x;   // mdp_solve_interface
    DevBuf rc_c, rc_w;                                          // mdp_reconstruct
};

// Grow-only device workspaces of a context.
struct Workspace {
    DevBuf a, b, c;       // folded batch buffers
    DevBuf zg;            // split-K partial products of the complex GEMM
    LSWork ls;            // interface least squares
    PackedWork pk;        // block-sparse interface matrix
    CallWork cw;          // per-call temporaries
    Profiler prof;        // optional per-launch timing
};

// Largest batch whose buffers fit in cap_bytes (at least 1, at most R).
int chunk_size(const APPlan& P, int precision, size_t cap_bytes, int R);

// Solve R auxiliary problems with right-hand sides described by src and hand
// the folded result to consume(u, du) (see solve_batch_t).
void solve_batch(const APPlan& P, Workspace& ws, int precision, const SrcDesc& src, bool src_cplx, int R,
                 const std::function<void(const void*, const float*)>& consume, hipStream_t st);

}  // namespace mdp
