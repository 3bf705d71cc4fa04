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
    // fused projector sweep, interleaved complex [(n+1)][W], scaled by the mode's off-diagonal a:
    DevBuf rf64;          // a r_m (r_m = 1/d'_m)
    DevBuf tf64;          // a tw_m (twisted pivots: sweep stopped at row m, zero right-hand side below)
    DevBuf rf32, tf32;    // FP32 copies of rf64, tf64
    std::vector<double> twist_ratio;   // per row m: smallest |1/tw_m| / row scale over all modes
    APPlan(int n, double h, double k);
};

// Least-squares buffers (grow-only).
// Pinned host memory for small device-to-host reads (grow-only; every read is
// followed by a wait for its stream, so a regrowth never frees memory a copy uses).
struct HostPinned {
    void* p = nullptr;
    size_t bytes = 0;
    HostPinned() = default;
    HostPinned(const HostPinned&) = delete;
    HostPinned& operator=(const HostPinned&) = delete;
    ~HostPinned() { if (p) (void)hipHostFree(p); }
    void* get(size_t b) {
        if (b > bytes) {
            if (p) MDP_HIP(hipHostFree(p));
            p = nullptr;
            bytes = 0;
            MDP_HIP(hipHostMalloc(&p, b, hipHostMallocDefault));
            bytes = b;
        }
        return p;
    }
};

struct LSWork {
    DevBuf G, L, Linv[3], T, A0, Aq, vec, norms, flags;
    DevBuf rp;           // refinement: per 32-row slab partial sums of A^* r (packed route)
    HostPinned hflags;   // the flags' host copy
};

// Packed interface matrix buffers (grow-only).
struct PackedWork {
    DevBuf Ap;
    DevBuf mf;            // multifrontal factor arena
};

// Interface assembly and reconstruction buffers (grow-only).
struct CallWork {
    DevBuf F, x;          // mdp_solve_interface
    DevBuf srcw;          // mdp_solve_interface: densities Ex^(I) f of the source right-hand sides
    DevBuf grad;          // mdp_dd_gradient: grids, vectors and tables of the reverse pass
    DevBuf jobs;          // job tables of batched launches across plans
};

// Grow-only device workspaces of a context.
struct Workspace {
    DevBuf a, b, c;       // folded batch buffers
    DevBuf zg;            // split-K partial products of the complex GEMM
    LSWork ls;            // interface least squares
    PackedWork pk;        // block-sparse interface matrix
    CallWork cw;          // per-call temporaries
    Staging stage;        // per-call descriptor uploads
    Profiler prof;        // optional per-launch timing
};

// Largest batch whose buffers fit in cap_bytes (at least 1, at most R).
int chunk_size(const APPlan& P, int precision, size_t cap_bytes, int R);

// Solve R auxiliary problems with right-hand sides described by src over the
// rows of band bd (exact when the right-hand side vanishes outside it; the full
// grid for a general one) and hand the folded result to consume(u, du, band)
// (see solve_batch_t; the refined precision always solves the full grid).
void solve_batch(const APPlan& P, Workspace& ws, int precision, const SrcDesc& src, bool src_cplx, int R, Band bd,
                 const std::function<void(const void*, const float*, Band)>& consume, hipStream_t st);

// Bytes of batch buffers a full-grid solve of R right-hand sides needs (solve_batch_scratch).
size_t solve_scratch_bytes(const APPlan& P, int precision, int R);
// The full-grid solve of solve_batch with its batch buffers in `scratch` (at least
// solve_scratch_bytes bytes, device): no workspace growth, no per-launch profiling, no
// GEMM autotuning, so nothing is allocated.
void solve_batch_scratch(const APPlan& P, int precision, void* scratch, const SrcDesc& src, bool src_cplx, int R,
                         const std::function<void(const void*, const float*, Band)>& consume, hipStream_t st);

// The library's static device scratch array of the allocation-free entry point: its
// size, and its address on `device` (resolved once per device; set-up call).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
void* noalloc_scratch(int device);

}  // namespace mdp
