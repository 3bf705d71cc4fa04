/*
 * mdp.h -- C-ABI of the MI355X (gfx950) library for the hot path of the
 * Method of Difference Potentials (MDP) applied to non-overlapping domain
 * decomposition of the Helmholtz equation
 *     Delta u + k^2 u = f  in Omega,   alpha u + beta du/dn = phi  on dOmega
 * (North, Tsynkov & Turkel, Sec. 3, eq. helmholtz_physical).
 *
 * The three calls follow the algorithm summary of Sec. 3.5:
 *   step 1b  mdp_build_projector  -- Q^(i) = [(P_gamma - I) Ex Psi_j], one
 *                                    auxiliary-problem (AP) solve per column;
 *   step 2   mdp_solve_interface  -- boundary and interface conditions
 *                                    eliminated in coefficient space, least
 *                                    squares for the coefficients c (with
 *                                    step 1c, the source's right-hand side F,
 *                                    when a source f is given);
 *   step 3   mdp_reconstruct      -- u = P_{N+} Ex(c) (+ G B f) on each subdomain.
 * mdp_ap_solve exposes G^(h), the AP solve itself (Sec. 3.2.1), on a batch of
 * right-hand sides.
 *
 * Conventions common to every call
 *   - Every function returns an mdp_status (0 = success).  On failure nothing
 *     has been launched and mdp_last_error(ctx) describes the cause; no C++
 *     exception crosses this interface.
 *   - "device" pointers are HIP device allocations on the context's device;
 *     "host" pointers are ordinary host memory.  Output buffers are owned by
 *     the caller; handles (mdp_ctx, mdp_projector) are owned by the library.
 *   - stream is a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Work is enqueued asynchronously on it unless stated otherwise.
 *   - Complex numbers are interleaved (re, im) FP64 pairs.
 *   - Grids: n cells per direction of the auxiliary square (n even, n >= 8);
 *     node (m, q), m, q = 0..n, sits at x = xa + m h, y = ya + q h with
 *     h = side/n.  A grid function is stored as (n+1)*(n+1) values, index
 *     m*(n+1) + q (x-major, y fastest).
 *   - Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef MDP_H
#define MDP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } mdp_c128;

typedef enum {
    MDP_OK = 0,
    MDP_ERR_ARG = -1,        /* invalid argument (sizes, null pointers, topology) */
    MDP_ERR_HIP = -2,        /* a HIP runtime call failed */
    MDP_ERR_OOM = -3,        /* device allocation failed */
    MDP_ERR_SINGULAR = -4,   /* an AP mode pivot or the interface factor broke down */
    MDP_ERR_NONFINITE = -5,  /* non-finite input data */
    MDP_ERR_NODEVICE = -6    /* no HIP device / bad device index */
} mdp_status;

/* Arithmetic of the AP solves.  The interface least squares is FP64 always. */
typedef enum {
    MDP_C128 = 0,         /* complex FP64 throughout */
    MDP_C64 = 1,          /* complex FP32 AP solves (FP32 MFMA, FP32 accumulation) */
    MDP_C64_REFINED = 2   /* FP32 solve + one FP64 residual and FP32 correction solve */
} mdp_precision;

/* How mdp_build_projector computes Q.  Both routes give the same Q up to
 * rounding order.
 * MDP_PATH_AUTO: for MDP_C128 and MDP_C64, the support-in / gamma-out route: the
 *   right-hand side L^(h) w |_{M+} lives on the two outer rings of M+ and
 *   only Tr_gamma of the AP solution is needed (eq. def_Pgamma), so only the
 *   four dense RHS rows and the four full gamma rows go through the sine
 *   GEMM; the other rows are transformed and synthesised inside one fused
 *   tridiagonal sweep that keeps the columns on chip.  Other precisions, and
 *   M+ boxes not symmetric about the AP centre line, use the dense route.
 * MDP_PATH_DENSE: every column is a full AP solve (sine GEMM of every grid
 *   row, tridiagonal solve, inverse GEMM) followed by the gather onto gamma. */
typedef enum {
    MDP_PATH_AUTO = 0,
    MDP_PATH_DENSE = 1
} mdp_projector_path;

/* How mdp_solve_interface solves the reduced least-squares system (steps 2b-2c
 * of Sec. 3.5).  Both use the normal equations of the column-equilibrated Qbar
 * with iterative refinement against the true residual (corrected semi-normal
 * equations); they differ in how the Gram matrix Qbar^* Qbar is factored.
 * MDP_IFACE_AUTO: dense up to 4096 unknowns, multifrontal above.
 * MDP_IFACE_DENSE: one dense blocked Cholesky of the Gram matrix and its inverse
 *   (order 4 n_sub M*; memory and work grow with its square and cube), with a
 *   Cholesky-QR fallback on the assembled Qbar for ill-conditioned systems.
 * MDP_IFACE_MULTIFRONTAL: nested dissection over the subdomain layout: the
 *   subdomains are halved recursively along the longer extent of their centres;
 *   each tree node eliminates the unknowns shared by its two halves (a dense
 *   partial Cholesky of its front) and passes the Schur complement on the
 *   unknowns it shares with the rest to its parent.  No dense fallback. */
typedef enum {
    MDP_IFACE_AUTO = 0,
    MDP_IFACE_DENSE = 1,
    MDP_IFACE_MULTIFRONTAL = 2
} mdp_interface_path;

/* One subdomain: the rectangle [x0, x0+lx] x [y0, y0+ly] with constant
 * wavenumber k (Sec. 3.1 assumes k constant on every subdomain).  Its
 * auxiliary domain is the square of side 1.1*max(lx, ly) centred on it, with
 * u = 0 on its top and bottom sides and the Sommerfeld-type conditions
 * u_x +- i k u = 0 on its left and right sides (eq. auxiliary_problem). */
typedef struct {
    double x0, y0, lx, ly;
    double k;
    int n;
} mdp_subdomain;

/* One side of one subdomain; sides are numbered 0 bottom, 1 top, 2 left, 3 right. */
typedef struct {
    int kind;              /* 0 = outer boundary, 1 = interface */
    double alpha, beta;    /* boundary: alpha u + beta du/dn = phi, (alpha, beta) != (0, 0)
                              (eq. helmholtz_robin, Sec. 3.3.1; n = outward normal) */
    const mdp_c128* d;     /* boundary: host, M* Chebyshev coefficients of phi in the side
                              parameter t (see mdp_cheb_coeffs); ignored for interfaces */
    int nbr, nbr_side;     /* interface: neighbouring subdomain and its side (Sec. 3.3.2);
                              the two sides must be the same segment */
} mdp_side;

typedef struct mdp_ctx mdp_ctx;
typedef struct mdp_projector mdp_projector;

/* Create a context on HIP device `device`.  *ctx receives the handle.
 * Errors: MDP_ERR_NODEVICE, MDP_ERR_HIP, MDP_ERR_ARG (ctx == NULL). */
int mdp_create(mdp_ctx** ctx, int device);

/* Destroy a context, its workspaces and its projector cache (projectors
 * still held by the caller stay valid until released). NULL is a no-op. */
void mdp_destroy(mdp_ctx* ctx);

/* Select the projector route of later mdp_build_projector calls on ctx
 * (projectors already cached are not rebuilt).  Errors: MDP_ERR_ARG. */
int mdp_set_projector_path(mdp_ctx* ctx, int path);

/* Autotuning (enable != 0) of the sine transform's GEMM and of the fused
 * projector sweep: the first GEMM of every (precision, n, number of rows within
 * a factor of two) times each eligible tile shape (128x128, 128x64, 64x64
 * workgroup tiles) on its own operands, and the first fused sweep of every
 * (precision, widest n, batch size within a factor of two) times 1, 2 and 4
 * mode columns per lane (see mdp_set_fused_schedule; a schedule set there
 * takes precedence), each keeping the fastest for later calls; a first call
 * waits for its stream.  The choices are process-wide; results change only by
 * rounding.  Errors: MDP_ERR_ARG (ctx == NULL). */
int mdp_set_autotune(mdp_ctx* ctx, int enable);

/* Schedule of the fused projector sweep (the MDP_PATH_AUTO route of
 * mdp_build_projector(s), complex128 and complex64) for later builds on ctx:
 * cols_per_lane = 1, 2 or 4 mode columns swept side by side by each lane of a
 * wavefront (independent recurrences; one load of a factor row serves them all),
 * or 0 (the default) to choose per batch of columns: two when the batch has
 * enough columns to keep about two wavefronts per SIMD busy, else one; with
 * mdp_set_autotune on, the fastest of 1, 2 and 4 measured at first use per
 * (precision, widest n, batch size within a factor of two).  Results change
 * only by rounding (the synthesis sums of a row are added in another order).
 * Errors: MDP_ERR_ARG (ctx NULL or another value). */
int mdp_set_fused_schedule(mdp_ctx* ctx, int cols_per_lane);

/* Columns per lane the last fused projector build on ctx used (0: none yet, or ctx NULL). */
int mdp_fused_schedule_used(const mdp_ctx* ctx);

/* Select the interface least-squares route (mdp_interface_path) of later
 * mdp_solve_interface calls on ctx.  Errors: MDP_ERR_ARG. */
int mdp_set_interface_path(mdp_ctx* ctx, int path);

/* Message of the last failure on ctx (or of the last mdp_create failure when
 * ctx is NULL).  Valid until the next call on the same context. */
const char* mdp_last_error(const mdp_ctx* ctx);

/* Step 1b of Sec. 3.5: Q = [(P_gamma - I) Ex Psi^(0)_1..4M*, (P_gamma - I) Ex Psi^(1)_1..4M*]
 * (eq. Q_construction), where Psi_j are Chebyshev polynomials T_0..T_{M*-1}
 * on each side (Sec. 3.2.4, eq. Psi_def) and Ex is the equation-based
 * extension through rho^4 (Sec. 3.2.3, eqs. general_extension, cartesian_extension).
 * Column col = kind*4M* + side*M* + j (kind 0 Dirichlet, 1 Neumann).
 * Each column costs one AP solve (P_gamma is applied as
 * (P_gamma - I) xi = -Tr_gamma G^(h)(L^(h) w |_{M+}), eqs. Potential_def, def_Pgamma).
 * All 8M* solves run as one batch on `stream`.
 * Projectors are cached in the context by (lx, ly, n, k, M*, precision) and
 * reference counted: a cache hit returns the same handle with its count
 * raised (Sec. 3.5: Q is computed once per distinct wavenumber).
 * Errors: MDP_ERR_ARG (n odd or < 8, M* < 1, lx/ly <= 0, subdomain not inside
 * its AP interior), MDP_ERR_NONFINITE (k not finite or <= 0), MDP_ERR_SINGULAR
 * (an AP mode factor breaks down), MDP_ERR_OOM, MDP_ERR_HIP. */
int mdp_build_projector(mdp_ctx* ctx, const mdp_subdomain* sd, int m_star, int precision,
                        void* stream, mdp_projector** out);

/* Step 1b for `count` subdomains at once (sds: host array), e.g. every
 * subdomain of a layout with uneven n and k: out[i] (host array of count
 * handles) receives subdomain i's projector, exactly as count calls of
 * mdp_build_projector would (same cache, same reference counts; subdomains
 * with equal (lx, ly, n, k) share one build).  On the MDP_PATH_AUTO route the
 * columns of every projector not yet cached run through the fused sweep
 * together: one launch per stage over all of them, the sine GEMMs one launch
 * per distinct n.  On failure no handle is returned (out[] is zeroed) and the
 * projectors built by the call stay in the cache.  Errors: as
 * mdp_build_projector, plus MDP_ERR_ARG for count < 1. */
int mdp_build_projectors(mdp_ctx* ctx, int count, const mdp_subdomain* sds, int m_star, int precision,
                         void* stream, mdp_projector** out);

/* Read-only view of a projector.  n_gamma = |gamma|; gamma_mq (host, 2*n_gamma
 * ints) lists gamma nodes as (m, q) pairs in increasing lexicographic (m, q)
 * order; q_dev (device, n_gamma x 8M* complex, column-major, leading
 * dimension n_gamma) is Q.  Any output pointer may be NULL.  The views stay
 * valid while the projector is held.  Errors: MDP_ERR_ARG (P == NULL). */
int mdp_projector_info(const mdp_projector* P, int* n_gamma, const int** gamma_mq,
                       const mdp_c128** q_dev);

/* Foot points of gamma for the source data of mdp_source: for gamma node i
 * (order of mdp_projector_info) on side s of the rectangle sd (the subdomain
 * the projector serves; it may sit anywhere), xy_out[2i], xy_out[2i+1] is the
 * point of the side's line at the node's side parameter (the node projected
 * onto the line, not clamped to the side) and side_out[i] = s (0 bottom,
 * 1 top, 2 left, 3 right; outward normal of that side).  Host arrays of
 * 2*n_gamma doubles and n_gamma ints; side_out may be NULL.
 * Errors: MDP_ERR_ARG (null pointers, sd of another size). */
int mdp_projector_gamma_feet(const mdp_projector* P, const mdp_subdomain* sd, double* xy_out, int* side_out);

/* Host helper: the auxiliary grid of the rectangle sd (Sec. 3.2.1; the square
 * of side 1.1*max(lx, ly) centred on it, n = sd->n cells per direction): node
 * (m, q) sits at (xa + m h, ya + q h).  Errors: MDP_ERR_ARG (null pointers,
 * non-positive or non-finite sizes, n odd or < 8). */
int mdp_ap_grid(const mdp_subdomain* sd, double* xa, double* ya, double* h);

/* Source f of Delta u + k^2 u = f on one subdomain (eq. helmholtz; Sec. 3.5
 * step 1c).  Device arrays, caller-owned, complex128:
 *   f    f at every node of the subdomain's auxiliary grid, (n+1)^2, index
 *        m*(n+1)+q (only the nodes of N+ are read), for the scheme's
 *        right-hand side B^(h) f (eq. rhs_g);
 *   jet  3*n_gamma: at the foot point of gamma node i (mdp_projector_gamma_feet),
 *        jet[i] = f, jet[n_gamma+i] = df/dn (outward normal),
 *        jet[2*n_gamma+i] = d2f/dn2 - d2f/dtau2, for the inhomogeneous part of
 *        the extension Ex^(I) f (eqs. cart_ext_2-4, extension_split).
 * A NULL f marks a subdomain without source. */
typedef struct {
    const mdp_c128* f;
    const mdp_c128* jet;
} mdp_source;

/* Drop one reference; the projector is freed with its last reference (the
 * context's cache holds one of its own until mdp_destroy or mdp_cache_clear).
 * Its device buffers go back to the context, whose later calls reuse them in
 * stream order after its earlier calls: device work of the caller's own that
 * reads Q must have completed when the last reference goes.  NULL is a no-op. */
void mdp_projector_release(mdp_projector* P);

/* Step 2 of Sec. 3.5.  subs (host, n_sub) are the subdomains; P[i] is
 * subdomain i's projector, built for a rectangle of the same size, n and k
 * (entries may alias: Q does not depend on the position of the rectangle);
 * sides is a host array of 4*n_sub entries, sides[4*i + s].  The boundary
 * conditions (eq. BC_coefficients) and interface conditions
 * (eq. transmission_coefficients) are resolved by elimination (Sec. 3.3.3),
 * giving the reduced system Qbar c = Fbar with sum|gamma_i| rows and
 * 4*n_sub*M* columns, which is solved in the least-squares sense (steps
 * 2b-2c) in FP64 on the device.  sources (host, n_sub entries, or NULL for
 * f = 0 everywhere) add each subdomain's right-hand side
 * F = (I - P_gamma) Ex^(I) f - Tr G^(h) B^(h) f (eq. linear_system_equations;
 * step 1c, one AP solve per subdomain with a source) to Fbar.
 * c_out (device, caller-owned, 8M* complex per subdomain, subdomain-major, each
 * in the column order of Q) receives every coefficient, known and solved.
 * rel_residual_out (host, may be NULL) = ||Qbar c - Fbar|| / ||Fbar||;
 * cond_estimate_out (host, may be NULL) estimates the 2-norm condition number
 * of the column-equilibrated Qbar.  The call waits for the least-squares
 * solve on `stream` (it returns host scalars); c_out is then written by work
 * queued on `stream`, so readers of c_out order themselves after the call on
 * `stream` (as mdp_reconstruct on the same stream does) or synchronise it.
 * Errors: MDP_ERR_ARG (inconsistent topology, mismatched interface segments,
 * alpha = beta = 0, M* or rectangle different from the projectors', null d),
 * MDP_ERR_NONFINITE, MDP_ERR_SINGULAR (the factor of Qbar broke down), MDP_ERR_OOM, MDP_ERR_HIP. */
int mdp_solve_interface(mdp_ctx* ctx, int n_sub, const mdp_subdomain* subs,
                        const mdp_projector* const* P, const mdp_side* sides, int m_star,
                        const mdp_source* sources, void* stream, mdp_c128* c_out, double* rel_residual_out,
                        double* cond_estimate_out);

/* Gradient of a receiver functional of the DD solve (f = 0) with respect to
 * every subdomain's k^2 and the boundary data, by a reverse pass through the
 * three steps of Sec. 3.5 (the conjugate-transposed AP solve of the
 * reconstruction, the adjoint of the coefficient expansion and of the least
 * squares, and k^2-directional derivatives of the AP solves: dA/dk^2 of the
 * scheme of eq. FD_scheme and of the x-end rows, dE/dk^2 of the extension of
 * eq. general_extension).  The functional is
 *     Phi = Re sum_t conj(ubar_t) u_{sub_t}(node_t),
 * u the reconstruction of mdp_reconstruct; for J = sum_t |u_t - u_obs_t|^2 pass
 * ubar = 2 (u - u_obs).  Arguments as mdp_solve_interface (the interface
 * system is solved again: nothing of an earlier call is kept); receivers (host
 * arrays of n_rcv): subdomain index, node index m*(n+1)+q of its auxiliary grid
 * (any node; the reconstruction is the solution on N+), complex weight ubar_t
 * (weights of one node add).  Outputs (host): grad_k2[i] = dPhi/d(k_i^2)
 * (n_sub doubles); grad_d[(4 i + s) M* + j] = dPhi/d(Re d) + i dPhi/d(Im d) for
 * coefficient j of boundary side s of subdomain i (zero for interface sides).
 * Requires complex128 projectors.  Waits for the stream.  Errors: as
 * mdp_solve_interface, plus MDP_ERR_ARG (receiver out of range, a projector
 * not complex128) and MDP_ERR_SINGULAR (the system needed the dense fallback). */
int mdp_dd_gradient(mdp_ctx* ctx, int n_sub, const mdp_subdomain* subs, const mdp_projector* const* P,
                    const mdp_side* sides, int m_star, int n_rcv, const int* rcv_sub, const int* rcv_node,
                    const mdp_c128* ubar, void* stream, double* grad_k2, mdp_c128* grad_d);

/* Step 3 of Sec. 3.5 for n_sub subdomains: xi_gamma = Ex(sum_j c_j Psi_j) and
 * u = P_{N+} xi_gamma = w - G^(h)(L^(h) w |_{M+}) (eqs. Potential_def,
 * potential_solution_homo); with sources (host, n_sub entries, or NULL),
 * xi_gamma also holds Ex^(I) f and u = P_{N+} xi_gamma + G^(h) B^(h) f =
 * w - G^(h)((L^(h) w - B^(h) f) |_{M+}) (eq. potential_solution).  c (device)
 * holds 8M* coefficients per subdomain
 * as written by mdp_solve_interface; u_out (device, caller-owned) receives
 * subdomain i's grid function at offset sum_{l<i} (n_l+1)^2 (complex); it is
 * the solution on N+, the difference potential at the other nodes of the grid
 * rows m_lo-1..m_hi+1 that hold N+ (the auxiliary solve stops at those rows:
 * its right-hand side vanishes outside them), and zero on the remaining rows.
 * Subdomains sharing a projector are solved in one batch, in the projector's
 * precision; when the subdomains use several projectors and no source is given,
 * all their solves run in the same launches in FP64 (whatever the projectors'
 * precision: that of a build refers to its 8M* solves per projector).
 * Errors: MDP_ERR_ARG, MDP_ERR_OOM, MDP_ERR_HIP. */
int mdp_reconstruct(mdp_ctx* ctx, int n_sub, const mdp_projector* const* P,
                    const mdp_c128* c, const mdp_source* sources, void* stream, mdp_c128* u_out);

/* G^(h) of Sec. 3.2.1 on `batch` right-hand sides: solves the discrete AP
 * (eq. discrete_AP: the compact scheme at interior nodes, u = 0 on q = 0, n,
 * fourth-order Sommerfeld-type rows at m = 0, n with zero right-hand side)
 * for g (device, batch grid functions; only interior nodes 1 <= m, q <= n-1
 * are read) into u (device, batch grid functions, zero on q = 0, n).
 * h = grid step, k = wavenumber.  Errors: MDP_ERR_ARG, MDP_ERR_NONFINITE,
 * MDP_ERR_SINGULAR, MDP_ERR_OOM, MDP_ERR_HIP. */
int mdp_ap_solve(mdp_ctx* ctx, int n, double h, double k, int precision, int batch,
                 const mdp_c128* g, mdp_c128* u, void* stream);

/* mdp_ap_solve without any device (or pinned host) allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and result as mdp_ap_solve (results
 * agree to rounding: the batch may be cut into chunks of another size, and the
 * sine GEMM always takes its default tile shape); the batch buffers live in a
 * library-owned static device array of 64 MiB per device (held by every device
 * the library runs on until the process ends) instead of the context's
 * workspaces; a batch larger than the array holds is solved in consecutive
 * chunks on `stream`.  Nothing in the array has to start at zero (each solve
 * writes every element it reads).  The plan of (n, h, k) must exist on ctx
 * already (an earlier mdp_ap_solve with the same n, h, k, e.g. with batch 0,
 * creates it); per-launch profiling and autotuning do not apply to this call.
 * All calls on one device share its array: calls that overlap in time on one
 * device race (order them on one stream, or synchronise between them).
 * Errors: MDP_ERR_ARG (no plan for (n, h, k), null pointers, one right-hand
 * side needing more than the 64 MiB: 32 (n+1) W bytes in complex128, 16 (n+1) W
 * in complex64, 24 (n+1) W refined, W the folded width of n, i.e. n/2 and
 * n/2 - 1 each rounded up to a multiple of 64: n = 1024 fits in every precision,
 * n = 2048 only in complex64), MDP_ERR_NONFINITE, MDP_ERR_HIP. */
int mdp_ap_solve_noalloc(mdp_ctx* ctx, int n, double h, double k, int precision, int batch, const mdp_c128* g,
                         mdp_c128* u, void* stream);

/* Host helper (Sec. 3.3.1: phi expanded in the same basis): t[i] =
 * cos(pi (i + 1/2)/M*), i = 0..M*-1, the sample points of mdp_cheb_coeffs. */
int mdp_cheb_points(int m_star, double* t);

/* Host helper: coefficients d_j (j = 0..M*-1) of the polynomial of degree < M*
 * interpolating samples[i] = phi(t_i) at the points of mdp_cheb_points,
 * d_j = (2 - delta_j0)/M* sum_i phi(t_i) T_j(t_i).  Errors: MDP_ERR_ARG. */
int mdp_cheb_coeffs(int m_star, const mdp_c128* samples, mdp_c128* d);

/* Drop the context's own reference to every cached projector (projectors the
 * caller still holds stay valid) so that the next mdp_build_projector
 * recomputes Q.  AP plans (sine matrices, per-mode tridiagonal factors),
 * geometries and workspaces are kept.  Does not wait for the device.
 * Errors: MDP_ERR_ARG (ctx == NULL). */
int mdp_cache_clear(mdp_ctx* ctx);

/* Per-launch profiling of the context's kernels: while enabled, every kernel
 * launch of the hot path is bracketed by HIP events recorded on the stream it
 * runs on and tagged with its kernel class and the launch's algorithmic flops
 * and bytes.  enable != 0 starts (and clears) the record, 0 stops it.
 * Errors: MDP_ERR_ARG. */
int mdp_profile_enable(mdp_ctx* ctx, int enable);

/* Restrict the per-launch profiling to the kernel classes named in `classes`
 * (comma-separated, e.g. "chol_panel,ap_fused_f64,interface_ls"); NULL or ""
 * records every class again.  Fewer records mean fewer event pairs on the
 * stream while the profiled steps are timed.  Errors: MDP_ERR_ARG. */
int mdp_profile_select(mdp_ctx* ctx, const char* classes);

/* JSON summary of the records since the last enable, one entry per kernel
 * class: {"class": {"count": c, "total_ms": t, "flops": f, "bytes": b}, ...},
 * written to buf (host, NUL-terminated, at most buflen bytes).  Synchronises
 * the device.  Errors: MDP_ERR_ARG (null or too small buffer), MDP_ERR_HIP. */
int mdp_profile_report(mdp_ctx* ctx, char* buf, int buflen);

/* Library version string (static). */
const char* mdp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MDP_H */
