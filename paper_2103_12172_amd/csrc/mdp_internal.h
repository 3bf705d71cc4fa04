// Internal declarations of the MDP library (host orchestration + HIP kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mdp.h"

namespace mdp {

// ----------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MDP_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            throw ::mdp::Error(e_ == hipErrorOutOfMemory ? MDP_ERR_OOM : MDP_ERR_HIP,        \
                               std::string(#call) + ": " + hipGetErrorString(e_));           \
    } while (0)

// ----------------------------------------------------------------- device buffer
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t b) { alloc(b); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t b) {
        release();
        if (b == 0) return;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error(MDP_ERR_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
        }
        bytes = b;
    }
    // grow-only reallocation (contents are not preserved)
    void reserve(size_t b) { if (b > bytes) alloc(b); }
    void release() { if (p) (void)hipFree(p); p = nullptr; bytes = 0; }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ----------------------------------------------------------------- descriptor uploads
// The small host-built tables of one call (descriptors, index maps) are packed
// into one byte image, each item 256-byte aligned, and moved to the device by
// a single asynchronous copy from pinned host memory: copies from pageable
// memory are staged synchronously by the runtime, one round trip per table.
class HostBlob {
public:
    template <class T>
    size_t put(const T* p, size_t n) {
        const size_t off = (data_.size() + 255) / 256 * 256;
        data_.resize(off + std::max<size_t>(n, 1) * sizeof(T), 0);
        if (n) std::memcpy(data_.data() + off, p, n * sizeof(T));
        return off;
    }
    template <class T>
    size_t put(const std::vector<T>& v) { return put(v.data(), v.size()); }
    size_t size() const { return data_.size(); }
    const char* data() const { return data_.data(); }
    // rewrite v at an offset an earlier put of the same size returned
    template <class T>
    void put_at(size_t off, const std::vector<T>& v) {
        if (off + v.size() * sizeof(T) > data_.size()) throw Error(MDP_ERR_ARG, "table rewrite out of range");
        if (!v.empty()) std::memcpy(data_.data() + off, v.data(), v.size() * sizeof(T));
    }

private:
    std::vector<char> data_;
};

// Pinned host staging buffers and a grow-only device image for per-call tables.
// A pinned slot is rewritten only after the copy out of it has completed (its
// event); several slots rotate so that the host rarely waits for a copy queued
// behind earlier work, and a copy takes a free slot that is already large enough
// when there is one.  A slot that must grow keeps its old buffer until the
// context is destroyed: freeing pinned memory synchronises the device, which
// would make the host wait for all queued work in the middle of a call.  The
// device image is rewritten by a copy ordered on the stream after every earlier
// call's kernels.
struct Staging {
    struct Slot {
        void* host = nullptr;
        size_t cap = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
    };
    static constexpr int kSlots = 8;
    Slot slot[kSlots];
    int next = 0;
    std::vector<void*> retired;   // outgrown slot buffers, freed with the context
    DevBuf image;
    Staging() = default;
    Staging(const Staging&) = delete;
    Staging& operator=(const Staging&) = delete;
    ~Staging() {
        for (Slot& s : slot) {
            if (s.pending) (void)hipEventSynchronize(s.done);
            if (s.host) (void)hipHostFree(s.host);
            if (s.done) (void)hipEventDestroy(s.done);
        }
        for (void* p : retired) (void)hipHostFree(p);
    }
    // copy b to the device address dst on st
    void copy(void* dst, const HostBlob& b, hipStream_t st) { copy(dst, b.data(), b.size(), st); }
    // copy n bytes at src (host) to the device address dst on st
    void copy(void* dst, const char* src, size_t n, hipStream_t st) {
        if (!n) return;
        // a free slot (its last copy completed) large enough, else any free slot, else the next
        // one in turn (waited for)
        int pick = -1, fit = -1;
        for (int i = 0; i < kSlots; ++i) {
            const int k = (next + i) % kSlots;
            Slot& c = slot[k];
            if (c.pending && hipEventQuery(c.done) != hipSuccess) continue;
            c.pending = false;
            if (pick < 0) pick = k;
            if (c.cap >= n) { fit = k; break; }
        }
        if (fit >= 0) pick = fit;
        if (pick < 0) pick = next;
        next = (pick + 1) % kSlots;
        Slot& s = slot[pick];
        if (!s.done) MDP_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
        if (s.pending) MDP_HIP(hipEventSynchronize(s.done));
        s.pending = false;
        if (n > s.cap) {
            const size_t want = std::max<size_t>({n, 2 * s.cap, (size_t)1 << 20});
            void* h = nullptr;
            MDP_HIP(hipHostMalloc(&h, want, hipHostMallocDefault));
            if (s.host) retired.push_back(s.host);
            s.host = h;
            s.cap = want;
        }
        std::memcpy(s.host, src, n);
        MDP_HIP(hipMemcpyAsync(dst, s.host, n, hipMemcpyHostToDevice, st));
        MDP_HIP(hipEventRecord(s.done, st));
        s.pending = true;
    }
    // the device image, grown (after the device has drained) to hold at least `bytes`
    // (tables that hold addresses inside the image are written after this)
    char* image_for(size_t bytes) {
        if (bytes > image.bytes) {
            MDP_HIP(hipDeviceSynchronize());
            image.reserve(std::max(bytes, 2 * image.bytes));
        }
        return image.as<char>();
    }
    // the device image, grown as above to b's size, with b copied in
    char* upload(const HostBlob& b, hipStream_t st) {
        char* img = image_for(b.size());
        copy(img, b, st);
        return img;
    }
};

// ----------------------------------------------------------------- per-launch profiler
// When enabled, every kernel launch of the hot path is bracketed by HIP events
// recorded on its own stream, tagged with a kernel class and the launch's
// algorithmic flops and bytes (what the algorithm must compute and move, not
// what the implementation happens to).
struct Profiler {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
        double flops, bytes;
    };
    bool on = false;
    std::vector<std::string> only;   // classes to record (all when empty)
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    bool wants(const char* name) const {
        if (!on) return false;
        if (only.empty()) return true;
        for (const auto& o : only)
            if (o == name) return true;
        return false;
    }
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        MDP_HIP(hipEventCreate(&e));
        return e;
    }
    template <class F>
    void run(const char* name, hipStream_t st, double flops, double bytes, F&& f) {
        if (!wants(name)) { f(); return; }
        hipEvent_t a = get(), b = get();
        MDP_HIP(hipEventRecord(a, st));
        f();
        MDP_HIP(hipEventRecord(b, st));
        recs.push_back({name, a, b, flops, bytes});
    }
    void reset() {
        for (auto& r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
        recs.clear();
    }
    ~Profiler() {
        reset();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// ----------------------------------------------------------------- geometry (host)
// Auxiliary grid of one subdomain and its grid sets (paper Sec. 3.2.2).
struct Geometry {
    double x0, y0, lx, ly;      // subdomain rectangle
    int n;                      // cells per direction of the auxiliary square
    double L, h, xa, ya;        // side, step, lower-left corner of the AP square
    int m_lo, m_hi, q_lo, q_hi; // M+ = [m_lo, m_hi] x [q_lo, q_hi] (inclusive)
    int n_gamma;
    std::vector<int> gm, gq;    // gamma nodes, increasing (m, q)
    std::vector<int> side;      // side of each gamma node (0 bottom, 1 top, 2 left, 3 right)
    std::vector<double> rho;    // signed distance to that side (> 0 outside)
    std::vector<double> t;      // side parameter in [-1, 1] (unclamped)
    std::vector<double> slen;   // side length
    std::vector<int> gmq;       // interleaved (m, q) pairs, for the public view
};

Geometry make_geometry(double x0, double y0, double lx, double ly, int n);

// Extension matrix E = Ex^(H) Psi (|gamma| x 8M*, column-major, real FP64) on
// the device from the gamma nodes' side, rho, t and side length; E must be
// zeroed first (only each row's own-side columns are written).
// deriv = 1: the derivative dE/d(k^2) instead of E
void launch_extension(const int* side, const double* rho, const double* t, const double* slen, int ng, double k,
                      int m_star, double* E, hipStream_t st, int deriv = 0);
// One entry of a build's set-up (device pointers).  A geometry new to the context:
// meta_words 4-byte words of gamma node tables copied from the call's upload (src) to
// its buffer (meta), and its node -> gamma map gidx ((n+1)^2) written from gm, gq.
// A projector: E (ng x 8M, column-major) from side, rho, t, slen and k.  Fields of
// the other kind are zero / null.
struct GeomJob {
    const char* src;
    char* meta;
    long meta_words;
    const int *side, *gm, *gq;
    const double *rho, *t, *slen;
    int ng, n, M;
    double k;
    double* E;
    int* gidx;
};
// every entry's set-up in two launches (tables, E and the -1 fill; then the gamma scatter)
void launch_geom_setup(const GeomJob* jobs_dev, int count, int max_nodes, hipStream_t st);

// ----------------------------------------------------------------- folded sine layout
// For even n = 2p the type-I sine transform splits by the parity of the mode j:
// S(n-q, j) = (-1)^(j+1) S(q, j).  A grid row of n-1 interior values is stored
// "folded" as two column blocks:
//   block 1 (width P1 >= p):   e_q = g_q + g_{n-q} (q < p), e_p = g_p   <-> odd modes  j = 2c+1
//   block 2 (width P2 >= p-1): o_q = g_q - g_{n-q} (q < p)              <-> even modes j = 2(c-P1)+2
// and the transform is a block-diagonal product of the two blocks with the
// corresponding sine sub-matrices.  Padding columns are zero.
struct Fold {
    int n = 0, p = 0, P1 = 0, P2 = 0, W = 0;
    static Fold make(int n);
};

// ----------------------------------------------------------------- kernel launchers (kernels_*.hip)
struct StencilCoef { double c0, ce, cc; };
struct EndRowCoef { double wD, wD2, wA, wA2, k; };

struct APDevPlan;  // forward

// RHS sources of an AP batch (all evaluated in FP64)
// GRID: a given grid on the interior nodes (zero on the x-end rows); GRID_ALL:
// a given grid on every unknown row, the x-end rows included
enum class Src { GRID = 0, STENCIL_GRID = 1, STENCIL_E = 2, GRID_ALL = 3 };

struct SrcDesc {
    Src kind;
    const double* grid;   // GRID / STENCIL_GRID: complex interleaved grids, (n+1)^2 each, stride grid_stride (complex elems)
    long grid_stride;
    const long* goff;     // optional: grid b starts at goff[b] (complex elements) instead of b * grid_stride
    const double* const* fsrc;   // STENCIL_GRID, optional: per entry b the source f on the grid (complex,
                                 // (n+1)^2) or null; the right-hand side becomes L w - B f on M+
    const double* E;      // STENCIL_E: column-major |gamma| x ncols real
    int ldE;
    int col0;             // STENCIL_E: first column of this batch
    const int* gidx;      // (n+1)^2 map node -> gamma index or -1
    int m_lo, m_hi, q_lo, q_hi;  // M+ box (STENCIL_*)
};

// Rows r0..r0+nr-1 of the AP grid held by a folded batch buffer (all n+1 rows for a full solve).
struct Band {
    int r0, nr;
};

template <class T>
void launch_fold_rhs(const SrcDesc& s, int n, const Fold& f, StencilCoef sc, int R, bool cplx, Band bd, T* out,
                     hipStream_t st);
// may_tune = false: the default tile shape (the autotuner creates HIP events at first use)
template <class T>
void launch_gemm_bd(const T* A, const T* B, T* C, long M, const Fold& f, hipStream_t st, bool may_tune = true);
// process-wide: pick the sine GEMM's tile shape per (precision, n, rows) by timing at first use
void set_gemm_autotune(int on);
// fac: planes l.re, l.im, r.re, r.im, tw.re, tw.im, each (n+1) x W
template <class T>
void launch_tridiag(const T* in, int planes_in, T* out, const T* fac, const T* colc, int n, const Fold& f, int R,
                    Band bd, hipStream_t st);
void launch_residual(const SrcDesc& s, int n, const Fold& f, StencilCoef sc, EndRowCoef ec, int R, bool cplx_src,
                     const float* u32, float* r_out, hipStream_t st);

// ----------------------------------------------------------------- adjoint (receiver functional)
// grids[off[t]] = val[t] (complex), t < count; the grids are cleared beforehand
void launch_scatter_values(const long* off, const double* val, int count, double* grids, hipStream_t st);
// wbar_b(i) = ubar_b(gamma_i) - sum over the 3x3 neighbours r of gamma_i in M+ of c(r) lambda_b(r)
// (the transpose of L^(h) restricted to M+, applied to lambda and read on gamma); grids at goff[b]
void launch_gamma_adjoint(const double* ubar, const double* lambda, const long* goff, int R, int n, StencilCoef sc,
                          int m_lo, int m_hi, int q_lo, int q_hi, const int* gm, const int* gq, int ng, double* wbar,
                          long wbar_stride, hipStream_t st);
// cbar_b(col) = sum_i E(i, col) wbar_b(i)  (E real |gamma| x ncol, column-major); cbar at cidx[b] * ncol
void launch_et_apply(const double* E, int ng, int ncol, const double* wbar, long wbar_stride, int R, const int* cidx,
                     double* cbar, hipStream_t st);
// xbar[src[e]] += conj(coef[e]) cbar[e] (at most two contributions per unknown; xbar cleared beforehand)
void launch_expand_adj(int n, const int* src, const double2* coef, const double2* cbar, double2* xbar, hipStream_t st);
// out[t] = (cbar[eidx[t]] - sum_r conj(Q_t(r, kcol[t])) Fb[roff_t + r]) / div[t] for the known coefficients t
// (Q_t the projector of entry t's subdomain, |gamma| rows, ld = rows)
void launch_data_grad(int count, const double2* const* Q, const int* rows, const int* kcol, const long* roff,
                      const int* eidx, const double* div, const double2* cbar, const double2* Fb, double2* out,
                      hipStream_t st);
// h_b = -dA v_b + (dL w_b + L dw_b)|M+ on every unknown row (dA: the derivative of the AP operator with respect to
// k^2; dL, L: stencil weights dsc, sc); grids at goff[b]
void launch_jvp_rhs(const double* v, const double* w, const double* dw, const long* goff, int R, int n, double h,
                    double k, StencilCoef sc, StencilCoef dsc, int m_lo, int m_hi, int q_lo, int q_hi, double* out,
                    hipStream_t st);
// out[i] = sum_g [conj(Fb(r0 + g)) yf(gamma_g) - conj(r(r0 + g)) yz(gamma_g)]
//          + sum over the receivers of the subdomain conj(ubar) (dwf - yf) at their nodes
void launch_kappa_dot(const double* yf, const double* yz, const double* dwf, const int* gm, const int* gq, int ng,
                      int n, const double2* Fb, const double2* r, long r0, const long* rcv_node, const double* rcv_val,
                      int rcv_count, double2* out, hipStream_t st);
template <class T>
void launch_gather_q(const T* u, const float* du, int n, const Fold& f, Band bd, const int* gm, const int* gq, int ng,
                     int R, double* Q, int ldq, int col0, hipStream_t st);
template <class T>
// out = w - u (w given) or u on the grid rows `rows` (inside the buffer's band bd); grid b of w and
// out starts at boff[b] (complex elements) when boff is set, else at b * stride
void launch_unfold_grid(const T* u, const float* du, int n, const Fold& f, Band bd, Band rows, int R, const double* w,
                        long w_stride, double* out, long out_stride, const long* boff, hipStream_t st);
// w_b(gamma_i) (+)= Ex^(I) f = rho^2/2 f + rho^3/6 df/dn + rho^4/24 (d2f/dn2 - d2f/dtau2 - k^2 f) from the
// jet of entry b (3 x ng complex, null: entry skipped); grid b of w at woff[b] (complex elements)
void launch_source_extension(const double* rho, const int* gm, const int* gq, int ng, int n, double k,
                             const double* const* jet, int R, double* w, const long* woff, bool accumulate,
                             hipStream_t st);
// F[foff[b] + i] += u_b(gamma_i) (u in folded band layout, complex F)
template <class T>
void launch_gather_add(const T* u, int n, const Fold& f, Band bd, const int* gm, const int* gq, int ng, int R,
                       double* F, const long* foff, hipStream_t st);
// w_b(gamma_i) = sum over the Dirichlet and Neumann columns of gamma_i's side of E(i, col) c_b(col)
void launch_extend_density(const double* E, int ng, int ncol, const double* c, const int* cidx, int R, const int* gm,
                           const int* gq, const int* gside, int n, double* w, long w_stride, const long* woff,
                           hipStream_t st);

// projector build, support-in / gamma-out form (FP64 or FP32 storage and arithmetic)
constexpr int FUSED_K = 8;   // rows per recomputed segment of the fused tridiagonal sweep
// One projector's columns in a batched support-in / gamma-out build: global
// columns b0 .. b0+R-1 of the launches are its columns src.col0 .. src.col0+R-1.
// Buffers are the job's own (column 0 of the job at the pointer); jobs of one
// n hold consecutive spec / spec_hat / xs / us ranges so that one sine GEMM per
// n covers them.  Layouts: gc [R][n+1][4] ring table, spec / spec_hat [R][4][W]
// folded special rows, rf / tf [(n+1)][W] interleaved complex a r_m (r_m = 1/d'_m) and
// a tw_m (twisted pivots), a the mode's off-diagonal, ckpt [R][nseg][2][W], xs / us
// [R][2][4][W], thin [R][W/64][rows_pad][4].  The buffers and the plan tables
// hold elements of the build's arithmetic type (double, or float for complex64):
// the pointers are typed double* and reinterpreted by the kernels.  Sf, Si are the
// folded sine matrices, colc the per-column off-diagonal, in the same type.
struct FusedJob {
    SrcDesc src;
    StencilCoef sc;
    Fold f;
    int nseg, rows_pad, ng, ldq;
    int b0, R;
    int g0[3];   // first group of 1, 2, 4 consecutive columns (groups never span two jobs)
    const double *Sf, *Si, *rf, *tf, *colc;
    double *gc, *spec, *spec_hat, *ckpt, *xs, *thin, *us, *Q;
    const int *gm, *gq;
};
// jobs: device table sorted by b0; total = sum of R; max_*: largest per-job extents; T the
// storage and arithmetic type of the build (double or float)
// the ring tables and special rows of every column (one workgroup per column; max_n the largest n)
template <class T>
void launch_fold_ring_jobs(const FusedJob* jobs, int njobs, int total, int max_n, hipStream_t st);
// LDS of the fold of one column of a grid with n cells (its density spread over 12 (n+1) doubles),
// and the most a workgroup may take (the fused route needs n up to about 1700)
inline size_t fold_ring_lds_bytes(int n) { return (size_t)12 * (n + 1) * sizeof(double); }
constexpr size_t kFoldRingMaxLds = 160 * 1024;
// the fused sweep, lanes_cols (1, 2 or 4) mode columns per lane (or, with may_tune and the sweep
// autotuner on, the fastest of the three for this kind of batch), max_w the widest job's W,
// waves_one_col the batch's wavefront count at one column per lane; returns the columns per lane
// it used
// groups[lg]: the number of groups of 1 << lg consecutive columns of one job over all jobs
// (the jobs' g0[lg] are their first groups)
template <class T>
int launch_proj_sweep_jobs(const FusedJob* jobs, int njobs, int total, const long* groups, int max_w,
                           long waves_one_col, int lanes_cols, bool may_tune, hipStream_t st);
// process-wide: pick the fused sweep's columns per lane by timing at first use
void set_sweep_autotune(int on);
// sweep_cols: the columns per lane the sweep ran with (its thin-sum layout)
template <class T>
void launch_gather_q_fused_jobs(const FusedJob* jobs, int njobs, int total, int max_ng, int sweep_cols,
                                hipStream_t st);
bool fused_projector_supported(const Fold& f, int m_lo, int m_hi, int q_lo, int q_hi);

// One plan's entries in a batched FP64 band solve across plans (the reconstruction of
// subdomains with different n and k): global entries b0 .. b0+R-1 are the job's entries
// 0 .. R-1.  Right-hand side src (entry b's grid at src.goff[b]); rows bd; batch buffers A, B
// ([b][2][bd.nr][W], the job's own regions; jobs of one n hold consecutive regions so one
// sine GEMM per n covers them); the density step reads E (|gamma| x ncol), the gamma lists
// and the coefficient vector cidx[b] of c, and writes entry b's grid at src.goff[b].
struct SolveJob {
    SrcDesc src;
    StencilCoef sc;
    Fold f;
    Band bd;
    int b0, R;
    double *A, *B;
    const double *fac, *colc;
    const double* E;
    int ng, ncol;
    const int *gm, *gq, *gside, *cidx;
    int adjoint;          // 1: conjugate-transposed mode solves (all rows)
    double* out;          // set: the solution into these grids (entry b at ooff[b]); null: w - u in place
    const long* ooff;
};
// w_b(gamma) = E c_b on the entries' grids (cleared beforehand); c: every subdomain's coefficients
void launch_extend_density_jobs(const SolveJob* jobs, int njobs, int total, int max_ng, double* grids,
                                const double* c, hipStream_t st);
// the folded right-hand sides of every entry into its job's A
void launch_fold_rhs_jobs(const SolveJob* jobs, int njobs, int total, int max_w, int max_nr, hipStream_t st);
// the mode solves of every entry, B -> A
void launch_tridiag_jobs(const SolveJob* jobs, int njobs, int total, int max_w, hipStream_t st);
// grid_b = w_b - u_b on the band rows, in place, or (job.out set) out_b = u_b (u from the job's B)
void launch_unfold_jobs(const SolveJob* jobs, int njobs, int total, int max_n, int max_nr, double* grids,
                        hipStream_t st);
int fused_segments(int m_lo, int m_hi);   // segments of FUSED_K rows covering m = m_lo-1..m_hi+1
// interface least squares
// tri: 0 full; 1 lower-triangle tiles of C only; 2 op(B) upper triangular (skip its zero part)
void launch_zgemm(char opA, char opB, int m, int n, int k, double2 alpha, const double2* A, int lda,
                  const double2* B, int ldb, double2 beta, double2* C, int ldc, DevBuf& ws, hipStream_t st,
                  int tri = 0);
void launch_znorm2(int m, const double2* v, double* out, hipStream_t st);
void launch_znormalize(int n, double2* v, double* norm_out, hipStream_t st);
void launch_scale_cols_checked(double2* A, int m, int n, int lda, const double* s, int* flags, hipStream_t st);
// One block step of the blocked Cholesky factorisation G + shift I = L L^* and
// of Z = L^{-1} (W: nc x nc accumulator of the inverse, zero initially; L, Z
// zero initially): columns kb .. kb+wtot-1 split into nq mutually uncoupled
// diagonal sub-blocks, sub-block q = kb+off[q] .. kb+off[q+1]-1 (1..64 columns
// each).  The panel launch factors the sub-blocks, the panel of L below the
// step and the block rows of Z; the update launch applies the trailing Schur
// update and the inverse accumulation.
struct CholStepDev {
    static constexpr int kMaxQ = 64;
    int kb, nq, wtot;
    int off[kMaxQ + 1];
};
// diagonal sub-blocks of a step (L(q,q), Z(q,q) = L(q,q)^{-1}, breakdown to *info), then the
// slabs: L(i,q) for the rows below the step and the block rows Z(q,j), j < kb
void launch_chol_diag(const double2* G, int nc, const CholStepDev& sp, double shift, double2* L, double2* Z, int* info,
                      hipStream_t st);
void launch_chol_slabs(const double2* G, int nc, const CholStepDev& sp, double2* L, double2* Z, const double2* W,
                       hipStream_t st);
// One matrix's share of a batched Cholesky step: sub-block kb..kb+w-1 of the order-nc matrix G
// (ld nc), its factor L, the inverse Z and the inverse's accumulator W (ld nc, columns < the
// eliminated count); np = ceil((nc-kb-w)/32) row slabs, nz = ceil(kb/32) Z slabs.
// workgroups of the update after the step kb..kb+w-1 of an order-nc matrix: tile x tile tiles
// of the trailing lower part and of the inverse accumulation (columns < kb + w)
__host__ __device__ inline int chol_update_tiles(int nc, int kb, int w, int tile) {
    const int ntr = (nc - kb - w + tile - 1) / tile, nw = (kb + w + tile - 1) / tile;
    return ntr * (ntr + 1) / 2 + ntr * nw;
}
// the update takes 64 x 64 tiles from this many workgroups of that size on (four per CU)
constexpr long kUpdWideMin = 1024;
struct CholBatchEntry {
    double2 *G, *L, *Z, *W;
    int nc, kb, w, np, nz;
};
void launch_chol_diag_batched(const CholBatchEntry* ent, int count, int* info, hipStream_t st);
void launch_chol_slabs_batched(const CholBatchEntry* ent, int count, int max_roles, hipStream_t st);
void launch_chol_update_batched(const CholBatchEntry* ent, int count, int max_tiles64, long tiles64, int max_tiles32,
                                hipStream_t st);
// trailing Schur complement and inverse accumulation after the step kb .. kb+wtot-1
void launch_chol_update(double2* G, int nc, int kb, int wtot, const double2* L, const double2* Z, double2* W,
                        hipStream_t st);
void launch_assemble_qbar(const double2* const* Qsrc, const int* qld, int n_sub, const int* row_off, int total_rows,
                          const int4* colmap, const double2* coefs, int ncol, double2* Qbar, int ldq, hipStream_t st);
// c[e] = known[e] + coef[e] x[src[e]] (src[e] < 0: known value only), e < n
void launch_expand_coeffs(int n, const int* src, const double2* coef, const double2* known, const double2* x,
                          double2* c, hipStream_t st);
void launch_known_rhs(const double2* const* Qsrc, const int* qld, int n_sub, const int* row_off, int total_rows,
                      const int* kcol, const double2* kval, const int* koff, double2* F, hipStream_t st);
void launch_col_norms(const double2* A, int m, int n, int lda, double* out, hipStream_t st);
void launch_scale_cols(double2* A, int m, int n, int lda, const double* s, int invert, hipStream_t st);
void launch_fill(double* p, long n, double v, hipStream_t st);

// packed (block-sparse) interface matrix: device views of the per-subdomain blocks
struct PackedDevice {
    const double2* const* Q;
    const int* m;
    const long* off;
    const int* s;
    const int* pc_sub;
    const int* pc_p;
    const int* pc_gcol;
    const int4* pc_cols;
    const double2* pc_coef;
    const long* roff;
    const int* pc_start;   // first packed column of each subdomain
    const int* gc_start = nullptr;   // global column g: its packed columns gc_list[gc_start[g] .. gc_start[g+1]-1]
    const int* gc_list = nullptr;
};
// column equilibration of the packed blocks: norms2[g] += ||packed columns of g||^2 (read from
// Q), norms = sqrt(norms2) (zero / non-finite raise flag bits 1 / 2), then the blocks
// assembled with every column divided by its global column's norm
void launch_packed_colnorm2(const PackedDevice& d, int total_pc, double* norms2, hipStream_t st);
void launch_finalize_norms(int n, const double* norms2, double* norms, int* flags, hipStream_t st);
void launch_assemble_packed(const PackedDevice& d, int total_pc, int max_m, const double* norms, double2* Ap,
                            hipStream_t st);
void launch_packed_ahx(const PackedDevice& d, int total_pc, const double2* Ap, const double2* v, double2 alpha,
                       double2* y, hipStream_t st);
void launch_packed_ax(const PackedDevice& d, int n_sub, int max_m, int max_s, const double2* Ap, const double2* x,
                      double2 alpha, double2* r, hipStream_t st);
// workgroup tile of the batched Gram products
constexpr int kGramTile = 32;
// One batch entry of the Gram products A_b^* A_b (A_b: k x n, column-major, ld k):
// its split-K partials start at P + poff, its column map at gcol + gcol_off.
struct ZBatch {
    const double2* A;
    int n, k, kchunk, gcol_off;
    long poff;
};
// G(lower) += A_b^* A_b scattered through the column maps, all batch entries in
// two launches (split-K products, then reduction + scatter); P holds
// nsplit * sum_b n_b^2 partial entries; G must hold the other contributions or zero.
void launch_gram_batched(const ZBatch* zb_dev, int nb, int max_n, int max_k, int nsplit, double2* P, const int* gcol,
                         double2* G, int ldg, hipStream_t st);
// y = op(A) x for lower-triangular A (n x n, ld lda), op 'N' or 'C'; y overwritten, fixed summation order.
void launch_trmv_lower(char op, int n, const double2* A, int lda, const double2* x, double2* y, hipStream_t st);
// y = A^* v on the packed matrix, one entry per global column (d.gc_start / d.gc_list set), y overwritten.
void launch_packed_ahx_set(const PackedDevice& d, int nc, const double2* Ap, const double2* v, double2* y,
                           hipStream_t st);
// out = F + alpha A x on the stacked rows (F null: alpha A x); norms: += ||out||^2, ||F||^2; clr: two
// accumulators of a later kernel set to zero.
void launch_packed_axpy(const PackedDevice& d, int n_sub, int max_m, const double2* Ap, const double2* x,
                        double2 alpha, const double2* F, double2* out, double* norms, double* clr, hipStream_t st);
// One pass over the packed matrix for a refinement step: r = F - A x on the stacked rows (kept on
// chip, not written) and its products A^* r, as per 32-row slab partial sums in P (packed column
// pc, slab q at P[pc * ms + q], ms = ceil(max_m / 32)); then y = A^* r, one entry per global
// column, the partials summed in a fixed order.  max_s: the most packed columns of a subdomain
// (up to 256 the slab stays in registers between the two products).  clr as in launch_packed_axpy.
inline int packed_slabs(int max_m) { return (max_m + 31) / 32; }
void launch_packed_resid_ahx(const PackedDevice& d, int n_sub, int max_m, int max_s, int nc, const double2* Ap,
                             const double2* x, const double2* F, double2* P, double2* y, double* clr,
                             hipStream_t st);
// out = a - b (out may alias a or b)
void launch_zsub(int n, const double2* a, const double2* b, double2* out, hipStream_t st);
// x += dx; norms: += ||x||^2 (updated), ||dx||^2; clr as above.
void launch_zaxpy_norms(int n, const double2* dx, double2* x, double* norms, double* clr, hipStream_t st);
// Multifrontal Cholesky of the interface Gram matrix: one node of the
// elimination tree.  Its front holds e eliminated columns, then b boundary
// columns (global indices idx[0..f-1], f = e + b).  A leaf assembles its
// subdomain's Gram block (split-K partials at P + poff, order n, nsplit splits of
// pstride entries; spos maps front positions to the block's columns); an inner
// node assembles its two children's contribution blocks (inv0/inv1 map front
// positions to a child's boundary positions, -1 if absent; kpos0/kpos1 map the
// child's boundary positions to front positions).  Int tables are byte offsets
// into the call's device image; G, L, Z, W, z, cw are element offsets into the
// factor arena: G the front (f x f, ld f), factored in place over its first e
// columns (afterwards its lower block G(e:, e:) is the contribution
// F22 - L21 L21^*); L (f x e, ld f) the factor's columns, L21 = its rows e..f-1;
// Z (ld f) holds L11^{-1}; W the inverse's accumulator; z (e) and cw (b) the
// forward solve's values and contribution.
struct MFNodeDev {
    int e, b, f, leaf;
    int n, nsplit;
    long pstride, poff;
    long spos, inv0, inv1, kpos0, kpos1, idx;
    int kid0, kid1;
    long G, L, Z, W, z, cw;
};
// all fronts of the nodes list[0..count-1] (max_f: their largest order)
void launch_mf_assemble(const MFNodeDev* nodes, const int* list, int count, int max_f, const char* img,
                        const double2* P, double2* arena, hipStream_t st);
// substitutions of the listed nodes (one tree height; max_e, max_b over them): forward
// (in = y): z = Linv w_e, cw = w_b - L21 z; backward (out = x, read at the boundary
// columns, written at the eliminated ones): t = z - L21^* x_b, x_e = Linv^* t
void launch_mf_solve(const MFNodeDev* nodes, const int* list, int count, int max_e, int max_b, bool forward,
                     const char* img, double2* arena, const double2* in, double2* out, hipStream_t st);

void launch_diag_range(const double2* L, int n, int ld, double* out, hipStream_t st);

}  // namespace mdp
