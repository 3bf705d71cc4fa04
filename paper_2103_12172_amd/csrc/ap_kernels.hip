// Memory-bound kernels of the auxiliary-problem (AP) solve and of the
// projector / reconstruction steps.
//
// Data layout in HBM (one batch of R right-hand sides, n even, p = n/2):
//   folded rows  buf[((b*planes + pl)*nr + m - r0)*W + c]
//     b = right-hand side, pl = 0 (real) / 1 (imaginary) plane, m = r0..r0+nr-1
//     the x index (a band of rows, all n+1 of them for a full solve), c the
//     folded column (block 1: e_q or odd modes, block 2: o_q or even modes, see
//     Fold).  Columns are contiguous, so a wavefront walking m for 64
//     consecutive columns reads 64 consecutive elements per step.
//   grids        complex interleaved FP64, (n+1)^2 per function, index m*(n+1)+q.
#include <hip/hip_complex.h>

#include <map>
#include <mutex>

#include "ap_solver.h"
#include "mdp_internal.h"

namespace mdp {
namespace {

struct C64 { double re, im; };
__device__ inline C64 cadd(C64 a, C64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline C64 csub(C64 a, C64 b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline C64 cscale(C64 a, double s) { return {a.re * s, a.im * s}; }

// ------------------------------------------------------------------ RHS sources (FP64)
// Value of the right-hand side at node (m, q) of batch entry b.
struct SrcEval {
    SrcDesc d;
    int n;
    StencilCoef sc;

    __device__ inline C64 wgrid(int b, int m, int q) const {   // density / grid value (complex)
        const long base = d.goff ? d.goff[b] : (long)b * d.grid_stride;
        const double* g = d.grid + 2 * (base + (long)m * (n + 1) + q);
        return {g[0], g[1]};
    }
    __device__ inline double wE(int b, int m, int q) const {   // density of column col0+b (real)
        int gi = d.gidx[m * (n + 1) + q];
        return gi >= 0 ? d.E[(long)(d.col0 + b) * d.ldE + gi] : 0.0;
    }
    __device__ inline bool in_mplus(int m, int q) const {
        return m >= d.m_lo && m <= d.m_hi && q >= d.q_lo && q <= d.q_hi;
    }
    // L^(h) applied to the density at an M+ node (eq. FD_scheme, left-hand side)
    __device__ inline C64 stencil(int b, int m, int q) const {
        if (d.kind == Src::STENCIL_E) {
            double ce = wE(b, m + 1, q) + wE(b, m - 1, q) + wE(b, m, q + 1) + wE(b, m, q - 1);
            double cc = wE(b, m + 1, q + 1) + wE(b, m - 1, q + 1) + wE(b, m + 1, q - 1) + wE(b, m - 1, q - 1);
            return {sc.c0 * wE(b, m, q) + sc.ce * ce + sc.cc * cc, 0.0};
        }
        C64 e = cadd(cadd(wgrid(b, m + 1, q), wgrid(b, m - 1, q)), cadd(wgrid(b, m, q + 1), wgrid(b, m, q - 1)));
        C64 k = cadd(cadd(wgrid(b, m + 1, q + 1), wgrid(b, m - 1, q + 1)),
                     cadd(wgrid(b, m + 1, q - 1), wgrid(b, m - 1, q - 1)));
        C64 c = wgrid(b, m, q);
        return {sc.c0 * c.re + sc.ce * e.re + sc.cc * k.re, sc.c0 * c.im + sc.ce * e.im + sc.cc * k.im};
    }
    // B^(h) f at an M+ node (eq. rhs_g) from entry b's source grid
    __device__ inline C64 bsource(const double* fg, int m, int q) const {
        auto at = [&](int mm, int qq) -> C64 {
            const double* p = fg + 2 * ((long)mm * (n + 1) + qq);
            return {p[0], p[1]};
        };
        const C64 c = at(m, q);
        const C64 e = cadd(cadd(at(m + 1, q), at(m - 1, q)), cadd(at(m, q + 1), at(m, q - 1)));
        return {c.re + (e.re - 4.0 * c.re) / 12.0, c.im + (e.im - 4.0 * c.im) / 12.0};
    }
    // right-hand side g(m, q) of the AP at an interior node (zero on the end rows)
    __device__ inline C64 rhs(int b, int m, int q) const {
        if (d.kind == Src::GRID_ALL) return (q <= 0 || q >= n) ? C64{0.0, 0.0} : wgrid(b, m, q);
        if (m <= 0 || m >= n || q <= 0 || q >= n) return {0.0, 0.0};
        if (d.kind == Src::GRID) return wgrid(b, m, q);
        if (!in_mplus(m, q)) return {0.0, 0.0};
        C64 v = stencil(b, m, q);
        if (d.kind == Src::STENCIL_GRID && d.fsrc && d.fsrc[b]) v = csub(v, bsource(d.fsrc[b], m, q));
        return v;
    }
};

// ------------------------------------------------------------------ fold RHS
// out row (b, m): block 1 col c = q-1 (q = 1..p):   e_q = g_q + g_{n-q} (e_p = g_p)
//                 block 2 col c = P1+q-1 (q < p):   o_q = g_q - g_{n-q}
template <class T>
__device__ inline void fold_rhs_body(const SrcEval& ev, const Fold& f, int planes, Band bd, T* __restrict__ out, int c,
                                     int m, int b) {
    const int n = f.n, p = f.p, W = f.W;
    C64 v = {0.0, 0.0};
    if (c < f.P1) {
        const int q = c + 1;
        if (q < p) v = cadd(ev.rhs(b, m, q), ev.rhs(b, m, n - q));
        else if (q == p) v = ev.rhs(b, m, p);
    } else {
        const int q = c - f.P1 + 1;
        if (q < p) v = csub(ev.rhs(b, m, q), ev.rhs(b, m, n - q));
    }
    const long o = (((long)b * planes) * bd.nr + (m - bd.r0)) * W + c;
    out[o] = (T)v.re;
    if (planes == 2) out[o + (long)bd.nr * W] = (T)v.im;
}

// Both folded entries that grid columns q and n - q feed, from one evaluation of each
// (column j < P1 of the odd-mode block: e_q, q = j + 1; column P1 + j < W of the even-mode
// block: o_q), and the zero padding of both blocks.
template <class T>
__device__ inline void fold_rhs_pair_body(const SrcEval& ev, const Fold& f, int planes, Band bd, T* __restrict__ out,
                                          int j, int m, int b) {
    const int n = f.n, p = f.p, W = f.W, q = j + 1;
    C64 e = {0.0, 0.0}, o = {0.0, 0.0};
    if (q < p) {
        const C64 g1 = ev.rhs(b, m, q), g2 = ev.rhs(b, m, n - q);
        e = cadd(g1, g2);
        o = csub(g1, g2);
    } else if (q == p) {
        e = ev.rhs(b, m, p);
    }
    const long o1 = (((long)b * planes) * bd.nr + (m - bd.r0)) * W + j;
    out[o1] = (T)e.re;
    if (planes == 2) out[o1 + (long)bd.nr * W] = (T)e.im;
    if (f.P1 + j < W) {
        const long o2 = o1 + f.P1;
        out[o2] = (T)o.re;
        if (planes == 2) out[o2 + (long)bd.nr * W] = (T)o.im;
    }
}

template <class T>
__global__ void __launch_bounds__(256)
fold_rhs_kernel(SrcEval ev, Fold f, int planes, Band bd, T* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= f.W) return;
    fold_rhs_body<T>(ev, f, planes, bd, out, c, bd.r0 + blockIdx.y, blockIdx.z);
}

// ------------------------------------------------------------------ tridiagonal solve per mode
// For column c (one sine mode) and right-hand side b, over the band of rows
// m = r0..t (t = r0 + nr - 1), Thomas with precomputed factors:
//   y_{r0-1} = 0, y_m = f_m - l_m y_{m-1};
//   x_t = tw_t y_t, x_m = r_m (y_m - s_m x_{m+1}) with s_0 = sup0 (complex end
//   row), s_m = a_c (interior off-diagonal) otherwise.
// For the full system (r0 = 0, t = n) this is the plain LU solve (tw_n = r_n).
// A band is exact when the right-hand side vanishes outside it: above it y is
// zero, below it the rows are eliminated in advance by the twisted pivot tw_t.
// fac planes: [0] l.re [1] l.im [2] r.re [3] r.im [4] tw.re [5] tw.im, each
// (n+1) x W by absolute row; colc: [0] a, [1] sup0.re, [2] sup0.im.
// y is kept in `out` between the sweeps.
// Conjugate-transposed solve T^H x = g for every mode column c and entry b, all
// rows m = 0..n, with the LU factors T = L U of the forward solve (L unit lower
// bidiagonal with l_m, U upper bidiagonal with pivots d_m = 1/r_m and
// super-diagonal s_m: s_0 = sup0, s_m = a):
//   U^H y = g:  y_m = conj(r_m) (g_m - conj(s_{m-1}) y_{m-1}),
//   L^H x = y:  x_n = y_n, x_m = y_m - conj(l_{m+1}) x_{m+1}.
// y is kept in `out` between the sweeps.  FP64, one column per thread.
__device__ inline void tridiag_adj_body(const double* __restrict__ in, int planes_in, double* __restrict__ out,
                                        const double* __restrict__ fac, const double* __restrict__ colc, int n, int W,
                                        int c, int b) {
    const long plane = (long)(n + 1) * W;
    const double* g_re = in + (long)b * planes_in * plane + c;
    const double* g_im = (planes_in == 2) ? g_re + plane : nullptr;
    double* o_re = out + (long)b * 2 * plane + c;
    double* o_im = o_re + plane;
    const double* l_re = fac + c;
    const double* l_im = fac + plane + c;
    const double* r_re = fac + 2 * plane + c;
    const double* r_im = fac + 3 * plane + c;
    const double a = colc[c], s0r = colc[W + c], s0i = colc[2 * W + c];
    // rows in groups of U with the next group's loads in flight
    constexpr int U = 8;
    double gr[U], gi[U], rr[U], ri[U], ngr[U], ngi[U], nrr[U], nri[U];
    auto load_fwd = [&](int m0, double* Gr, double* Gi, double* Rr, double* Ri) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long off = (long)min(m0 + u, n) * W;
            Gr[u] = g_re[off];
            Gi[u] = g_im ? g_im[off] : 0.0;
            Rr[u] = r_re[off];
            Ri[u] = r_im[off];
        }
    };
    double yr = 0.0, yi = 0.0;
    load_fwd(0, gr, gi, rr, ri);
    for (int m0 = 0; m0 <= n; m0 += U) {
        if (m0 + U <= n) load_fwd(m0 + U, ngr, ngi, nrr, nri);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = m0 + u;
            if (m > n) break;
            double xr_ = gr[u], xi_ = gi[u];
            if (m >= 1) {   // g - conj(s) y
                const double sr = (m == 1) ? s0r : a, si = (m == 1) ? s0i : 0.0;
                xr_ -= sr * yr + si * yi;
                xi_ -= sr * yi - si * yr;
            }
            yr = rr[u] * xr_ + ri[u] * xi_;   // conj(r) (g - conj(s) y)
            yi = rr[u] * xi_ - ri[u] * xr_;
            o_re[(long)m * W] = yr;
            o_im[(long)m * W] = yi;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            gr[u] = ngr[u];
            gi[u] = ngi[u];
            rr[u] = nrr[u];
            ri[u] = nri[u];
        }
    }
    // x_n = y_n; x_m = y_m - conj(l_{m+1}) x_{m+1}, rows n-1..0 in groups of U
    double xr = yr, xi = yi;
    auto load_bwd = [&](int mtop, double* Yr, double* Yi, double* Lr, double* Li) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = max(mtop - u, 0);
            Yr[u] = o_re[(long)m * W];
            Yi[u] = o_im[(long)m * W];
            Lr[u] = l_re[(long)(m + 1) * W];
            Li[u] = l_im[(long)(m + 1) * W];
        }
    };
    load_bwd(n - 1, gr, gi, rr, ri);
    for (int mtop = n - 1; mtop >= 0; mtop -= U) {
        if (mtop - U >= 0) load_bwd(mtop - U, ngr, ngi, nrr, nri);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = mtop - u;
            if (m < 0) break;
            const double nxr = gr[u] - (rr[u] * xr + ri[u] * xi);
            const double nxi = gi[u] - (rr[u] * xi - ri[u] * xr);
            xr = nxr;
            xi = nxi;
            o_re[(long)m * W] = xr;
            o_im[(long)m * W] = xi;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            gr[u] = ngr[u];
            gi[u] = ngi[u];
            rr[u] = nrr[u];
            ri[u] = nri[u];
        }
    }
}

template <class T>
__device__ __attribute__((always_inline)) inline void tridiag_body(const T* __restrict__ in, int planes_in, T* __restrict__ out,
                                    const T* __restrict__ fac, const T* __restrict__ colc, int n, int W, Band bd,
                                    int c, int b) {
    const int r0 = bd.r0, t = bd.r0 + bd.nr - 1;
    const long plane = (long)bd.nr * W, fplane = (long)(n + 1) * W;
    const T* fin_re = in + (long)b * planes_in * plane + c - (long)r0 * W;   // indexed by absolute row
    const T* fin_im = (planes_in == 2) ? fin_re + plane : nullptr;
    T* o_re = out + (long)b * 2 * plane + c - (long)r0 * W;
    T* o_im = o_re + plane;
    const T* l_re = fac + c;
    const T* l_im = fac + fplane + c;
    const T* r_re = fac + 2 * fplane + c;
    const T* r_im = fac + 3 * fplane + c;
    const T a = colc[c], s0r = colc[W + c], s0i = colc[2 * W + c];
    const T twr = fac[4 * fplane + (long)t * W + c], twi = fac[5 * fplane + (long)t * W + c];

    // forward sweep, rows in groups of U with the next group's loads in flight
    constexpr int U = 8;
    T yr = T(0), yi = T(0);
    T fr[U], fi[U], lr[U], li[U], nfr[U], nfi[U], nlr[U], nli[U];
    auto load_fwd = [&](int m0, T* F, T* Fi, T* Lr, T* Li) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long off = (long)min(m0 + u, t) * W;
            F[u] = fin_re[off];
            Fi[u] = fin_im ? fin_im[off] : T(0);
            Lr[u] = l_re[off];
            Li[u] = l_im[off];
        }
    };
    load_fwd(r0, fr, fi, lr, li);
    for (int m0 = r0; m0 <= t; m0 += U) {
        if (m0 + U <= t) load_fwd(m0 + U, nfr, nfi, nlr, nli);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = m0 + u;
            if (m > t) break;
            // y = f - l y_prev as two dependent fma per component (y_{r0-1} = 0, l_0 = 0)
            const T nr = fma(-lr[u], yr, fma(li[u], yi, fr[u]));
            const T ni = fma(-lr[u], yi, fma(-li[u], yr, fi[u]));
            yr = nr;
            yi = ni;
            o_re[(long)m * W] = yr;
            o_im[(long)m * W] = yi;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            fr[u] = nfr[u];
            fi[u] = nfi[u];
            lr[u] = nlr[u];
            li[u] = nli[u];
        }
    }
    // backward sweep over the same groups, last group first; y comes back from out
    T xr = T(0), xi = T(0);
    const int last = r0 + ((t - r0) / U) * U;
    auto load_bwd = [&](int m0, T* Yr, T* Yi, T* Qr, T* Qi) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = min(m0 + u, t);
            const long off = (long)m * W;
            Yr[u] = o_re[off];
            Yi[u] = o_im[off];
            Qr[u] = (m == t) ? twr : r_re[off];
            Qi[u] = (m == t) ? twi : r_im[off];
        }
    };
    load_bwd(last, fr, fi, lr, li);
    for (int m0 = last; m0 >= r0; m0 -= U) {
        if (m0 - U >= r0) load_bwd(m0 - U, nfr, nfi, nlr, nli);
#pragma unroll
        for (int u = U - 1; u >= 0; --u) {
            const int m = m0 + u;
            if (m > t) continue;
            // x = rr (y - s x_next) = p - q x_next with p = rr y, q = rr s off the dependency chain
            // (x_{t+1} does not enter: xr = 0 there)
            const T sr = (m == 0) ? s0r : a, si = (m == 0) ? s0i : T(0);
            const T ppr = fma(lr[u], fr[u], -(li[u] * fi[u])), ppi = fma(lr[u], fi[u], li[u] * fr[u]);
            const T qr = fma(lr[u], sr, -(li[u] * si)), qi = fma(lr[u], si, li[u] * sr);
            const T nxr = fma(-qr, xr, fma(qi, xi, ppr));
            const T nxi = fma(-qr, xi, fma(-qi, xr, ppi));
            xr = nxr;
            xi = nxi;
            o_re[(long)m * W] = xr;
            o_im[(long)m * W] = xi;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            fr[u] = nfr[u];
            fi[u] = nfi[u];
            lr[u] = nlr[u];
            li[u] = nli[u];
        }
    }
}

template <class T>
__global__ void __launch_bounds__(256)
tridiag_kernel(const T* __restrict__ in, int planes_in, T* __restrict__ out, const T* __restrict__ fac,
               const T* __restrict__ colc, int n, int W, int R, Band bd) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= W || b >= R) return;
    tridiag_body<T>(in, planes_in, out, fac, colc, n, W, bd, c, b);
}

// The same solve cut into P row segments, one wavefront each (64 columns per
// workgroup), for batches too small to fill the chip one column per thread.
// Both sweeps are first-order linear recurrences,
//   y_m = f_m - l_m y_{m-1},   x_m = rr_m y_m - rr_m s_m x_{m+1}   (rr_t = tw_t),
// so each segment runs its recurrence from a zero start together with the
// product of its coefficients (phi = prod(-l_m) forward, psi = prod(-rr_m s_m)
// backward), one wavefront chains the P segment ends in order, and every
// segment then adds phi (psi) times the value carried into it.  The rounding
// is that of the sequential sweep: the same products of l (r s) multiply the
// same terms, only grouped by segment.
template <class T>
struct PartLds {
    T er[16][64], ei[16][64];   // segment end values (zero-start run)
    T pr[16][64], pi[16][64];   // segment coefficient products
    T cr[16][64], ci[16][64];   // values carried into the segments
};

template <class T>
__global__ void __launch_bounds__(1024)
tridiag_part_kernel(const T* __restrict__ in, int planes_in, T* __restrict__ out, const T* __restrict__ fac,
                    const T* __restrict__ colc, int n, int W, Band bd, int P, int Lseg) {
    __shared__ PartLds<T> s;
    const int lane = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane, b = blockIdx.y;
    const bool act = c < W && p < P;
    const int r0 = bd.r0, t = bd.r0 + bd.nr - 1;
    const int ms = r0 + p * Lseg, me = min(ms + Lseg - 1, t);
    const long plane = (long)bd.nr * W, fplane = (long)(n + 1) * W;
    const int cc = min(c, W - 1);
    const T* fin_re = in + (long)b * planes_in * plane + cc - (long)r0 * W;   // indexed by absolute row
    const T* fin_im = (planes_in == 2) ? fin_re + plane : nullptr;
    T* o_re = out + (long)b * 2 * plane + cc - (long)r0 * W;
    T* o_im = o_re + plane;
    const T* l_re = fac + cc;
    const T* l_im = fac + fplane + cc;
    const T* r_re = fac + 2 * fplane + cc;
    const T* r_im = fac + 3 * fplane + cc;
    const T a = colc[cc], s0r = colc[W + cc], s0i = colc[2 * W + cc];
    const T twr = fac[4 * fplane + (long)t * W + cc], twi = fac[5 * fplane + (long)t * W + cc];
    constexpr int U = 8;
    T vr[U], vi[U], kr[U], ki[U];   // per row of a group: data value and recurrence coefficient

    // forward group loads: data (from `src` planes) and -l_m
    auto load_f = [&](int g0, const T* sre, const T* sim) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long off = (long)min(g0 + u, me) * W;
            vr[u] = sre[off];
            vi[u] = sim ? sim[off] : T(0);
            kr[u] = -l_re[off];
            ki[u] = -l_im[off];
        }
    };
    // backward group loads: y_m and rr_m
    auto load_b = [&](int g0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int m = min(g0 + u, me);
            const long off = (long)m * W;
            vr[u] = o_re[off];
            vi[u] = o_im[off];
            kr[u] = (m == t) ? twr : r_re[off];
            ki[u] = (m == t) ? twi : r_im[off];
        }
    };
    const int glast = ms + ((me - ms) / U) * U;

    // A: forward run from zero and phi over the segment; the run goes to out
    T yr = T(0), yi = T(0), fr = T(1), fi = T(0);
    if (act) {
        for (int g0 = ms; g0 <= me; g0 += U) {
            load_f(g0, fin_re, fin_im);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (g0 + u > me) break;
                const T nr = fma(kr[u], yr, fma(-ki[u], yi, vr[u])), ni = fma(kr[u], yi, fma(ki[u], yr, vi[u]));
                const T qr = fma(kr[u], fr, -(ki[u] * fi)), qi = fma(kr[u], fi, ki[u] * fr);
                yr = nr; yi = ni; fr = qr; fi = qi;
                o_re[(long)(g0 + u) * W] = yr;
                o_im[(long)(g0 + u) * W] = yi;
            }
        }
        s.er[p][lane] = yr; s.ei[p][lane] = yi;
        s.pr[p][lane] = fr; s.pi[p][lane] = fi;
    }
    __syncthreads();
    if (p == 0) {   // y at the end of every segment, segment by segment
        T Yr = T(0), Yi = T(0);
        for (int q = 0; q < P; ++q) {
            const T pr = s.pr[q][lane], pi = s.pi[q][lane];
            const T nr = s.er[q][lane] + (pr * Yr - pi * Yi), ni = s.ei[q][lane] + (pr * Yi + pi * Yr);
            Yr = nr; Yi = ni;
            s.cr[q][lane] = Yr; s.ci[q][lane] = Yi;
        }
    }
    __syncthreads();
    // C: y_m = run_m + phi_m Y_in
    if (act) {
        const T Yr = (p > 0) ? s.cr[p - 1][lane] : T(0), Yi = (p > 0) ? s.ci[p - 1][lane] : T(0);
        fr = T(1); fi = T(0);
        for (int g0 = ms; g0 <= me; g0 += U) {
            load_f(g0, o_re, o_im);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (g0 + u > me) break;
                const T qr = fma(kr[u], fr, -(ki[u] * fi)), qi = fma(kr[u], fi, ki[u] * fr);
                fr = qr; fi = qi;
                o_re[(long)(g0 + u) * W] = fma(fr, Yr, fma(-fi, Yi, vr[u]));
                o_im[(long)(g0 + u) * W] = fma(fr, Yi, fma(fi, Yr, vi[u]));
            }
        }
    }
    __syncthreads();
    // D: backward run from zero and psi over the segment (the segment holding t starts with x_t = tw_t y_t)
    T xr = T(0), xi = T(0), gr = T(1), gi = T(0);
    if (act) {
        for (int g0 = glast; g0 >= ms; g0 -= U) {
            load_b(g0);
#pragma unroll
            for (int u = U - 1; u >= 0; --u) {
                const int m = g0 + u;
                if (m > me) continue;
                // x = p - q x_next with p = rr y, q = rr s (off the dependency chain); psi *= -q
                const T sr = (m == 0) ? s0r : a, si = (m == 0) ? s0i : T(0);
                const T ppr = fma(kr[u], vr[u], -(ki[u] * vi[u])), ppi = fma(kr[u], vi[u], ki[u] * vr[u]);
                const T qr = fma(kr[u], sr, -(ki[u] * si)), qi = fma(kr[u], si, ki[u] * sr);
                const T nxr = fma(-qr, xr, fma(qi, xi, ppr));
                const T nxi = fma(-qr, xi, fma(-qi, xr, ppi));
                xr = nxr; xi = nxi;
                const T hr = fma(-qr, gr, qi * gi), hi = fma(-qr, gi, -(qi * gr));
                gr = hr; gi = hi;
                o_re[(long)m * W] = xr;
                o_im[(long)m * W] = xi;
            }
        }
        s.er[p][lane] = xr; s.ei[p][lane] = xi;
        s.pr[p][lane] = gr; s.pi[p][lane] = gi;
    }
    __syncthreads();
    if (p == 0) {   // x at the start of every segment, last segment first
        T Xr = T(0), Xi = T(0);
        for (int q = P - 1; q >= 0; --q) {
            const T pr = s.pr[q][lane], pi = s.pi[q][lane];
            const T nr = s.er[q][lane] + (pr * Xr - pi * Xi), ni = s.ei[q][lane] + (pr * Xi + pi * Xr);
            Xr = nr; Xi = ni;
            s.cr[q][lane] = Xr; s.ci[q][lane] = Xi;
        }
    }
    __syncthreads();
    // F: x_m = run_m + psi_m X_in
    if (act) {
        const T Xr = (p + 1 < P) ? s.cr[p + 1][lane] : T(0), Xi = (p + 1 < P) ? s.ci[p + 1][lane] : T(0);
        gr = T(1); gi = T(0);
        for (int g0 = glast; g0 >= ms; g0 -= U) {
            load_b(g0);   // vr/vi: the backward run
#pragma unroll
            for (int u = U - 1; u >= 0; --u) {
                const int m = g0 + u;
                if (m > me) continue;
                const T sr = (m == 0) ? s0r : a, si = (m == 0) ? s0i : T(0);
                const T qr = fma(kr[u], sr, -(ki[u] * si)), qi = fma(kr[u], si, ki[u] * sr);
                const T hr = fma(-qr, gr, qi * gi), hi = fma(-qr, gi, -(qi * gr));
                gr = hr; gi = hi;
                o_re[(long)m * W] = fma(gr, Xr, fma(-gi, Xi, vr[u]));
                o_im[(long)m * W] = fma(gr, Xi, fma(gi, Xr, vi[u]));
            }
        }
    }
}

// ------------------------------------------------------------------ unfold helpers
// u(m, q) of right-hand side b, plane pl, from folded synthesis rows:
//   u_q = A_q + B_q, u_{n-q} = A_q - B_q (q < p), u_p = A_p, zero at q = 0, n.
template <class T>
__device__ inline double unfold_at(const T* __restrict__ u, const Fold& f, Band bd, int b, int pl, int m, int q) {
    const int n = f.n, p = f.p;
    if (q <= 0 || q >= n) return 0.0;
    const T* row = u + (((long)b * 2 + pl) * bd.nr + (m - bd.r0)) * f.W;
    if (q == p) return (double)row[p - 1];
    if (q < p) return (double)row[q - 1] + (double)row[f.P1 + q - 1];
    const int qq = n - q;
    return (double)row[qq - 1] - (double)row[f.P1 + qq - 1];
}

template <class T>
__device__ inline C64 unfold_c(const T* __restrict__ u, const Fold& f, Band bd, int b, int m, int q) {
    return {unfold_at(u, f, bd, b, 0, m, q), unfold_at(u, f, bd, b, 1, m, q)};
}

// ------------------------------------------------------------------ residual (refinement)
// r = g - A u32 over every row of the discrete AP, in FP64, directly in folded
// coordinates.  The folded synthesis rows hold A_q = (u_q + u_{n-q})/2 and
// B_q = (u_q - u_{n-q})/2; every row of the AP is symmetric under q -> n-q, so
//   r_q + r_{n-q} = (g_q + g_{n-q}) - 2 (Op A)_q   (q < p),  r_p = g_p - (Op A)_p,
//   r_q - r_{n-q} = (g_q - g_{n-q}) - 2 (Op B)_q   (q < p),
// where Op is the interior 9-node stencil (1 <= m <= n-1) or the Sommerfeld-type
// end row (m = 0, n), applied to the A block extended evenly about q = p
// (A_0 = 0, A_{p+1} = A_{p-1}) or to the B block extended oddly (B_0 = B_p = 0).
// Output: the folded residual as FP32 real/imaginary planes.
struct FoldedField {
    const float* __restrict__ u;
    Fold f;
    // value of plane pl of the even (blk 0) or odd (blk 1) field at (m, q), q = 0..p+1
    __device__ inline double at(int b, int pl, int m, int q, int blk) const {
        const int p = f.p;
        const float* row = u + (((long)b * 2 + pl) * (f.n + 1) + m) * f.W;
        if (blk == 0) {
            if (q <= 0) return 0.0;
            if (q > p) q = 2 * p - q;
            return (double)row[q - 1];
        }
        if (q <= 0 || q >= p) {
            if (q > p) return -(double)row[f.P1 + (2 * p - q) - 1];
            return 0.0;
        }
        return (double)row[f.P1 + q - 1];
    }
    __device__ inline C64 atc(int b, int m, int q, int blk) const { return {at(b, 0, m, q, blk), at(b, 1, m, q, blk)}; }
};

__global__ void __launch_bounds__(256)
residual_kernel(SrcEval ev, EndRowCoef ec, Fold f, const float* __restrict__ u32, float* __restrict__ r_out) {
    const int n = f.n, p = f.p, W = f.W;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y, b = blockIdx.z;
    if (c >= W) return;
    const FoldedField F{u32, f};
    int blk, q;
    if (c < f.P1) { blk = 0; q = c + 1; if (q > p) q = -1; }
    else { blk = 1; q = c - f.P1 + 1; if (q >= p) q = -1; }
    C64 r = {0.0, 0.0};
    if (q > 0) {
        // folded right-hand side
        C64 g;
        if (blk == 0) g = (q < p) ? cadd(ev.rhs(b, m, q), ev.rhs(b, m, n - q)) : ev.rhs(b, m, p);
        else g = csub(ev.rhs(b, m, q), ev.rhs(b, m, n - q));
        const double wgt = (blk == 0 && q == p) ? 1.0 : 2.0;
        C64 op;
        if (m > 0 && m < n) {
            const StencilCoef sc = ev.sc;
            C64 e = cadd(cadd(F.atc(b, m + 1, q, blk), F.atc(b, m - 1, q, blk)),
                         cadd(F.atc(b, m, q + 1, blk), F.atc(b, m, q - 1, blk)));
            C64 k = cadd(cadd(F.atc(b, m + 1, q + 1, blk), F.atc(b, m - 1, q + 1, blk)),
                         cadd(F.atc(b, m + 1, q - 1, blk), F.atc(b, m - 1, q - 1, blk)));
            C64 cc = F.atc(b, m, q, blk);
            op = {sc.c0 * cc.re + sc.ce * e.re + sc.cc * k.re, sc.c0 * cc.im + sc.ce * e.im + sc.cc * k.im};
        } else {
            // D = u(m_out) - u(m_in), A = (u(m_out) + u(m_in))/2 at q-1, q, q+1; +- i k on the A part
            const int mo = (m == 0) ? 1 : n, mi = (m == 0) ? 0 : n - 1;
            const double sgn = (m == 0) ? -1.0 : 1.0;
            C64 D[3], Av[3];
            for (int t = 0; t < 3; ++t) {
                C64 uo = F.atc(b, mo, q + t - 1, blk), ui = F.atc(b, mi, q + t - 1, blk);
                D[t] = csub(uo, ui);
                Av[t] = cscale(cadd(uo, ui), 0.5);
            }
            C64 d2D = cadd(csub(D[2], cscale(D[1], 2.0)), D[0]);
            C64 d2A = cadd(csub(Av[2], cscale(Av[1], 2.0)), Av[0]);
            C64 dpart = cadd(cscale(D[1], ec.wD), cscale(d2D, ec.wD2));
            C64 apart = cadd(cscale(Av[1], ec.wA), cscale(d2A, ec.wA2));
            op = {dpart.re - sgn * ec.k * apart.im, dpart.im + sgn * ec.k * apart.re};
        }
        r = {g.re - wgt * op.re, g.im - wgt * op.im};
    }
    const long o = (((long)b * 2) * (n + 1) + m) * W + c;
    r_out[o] = (float)r.re;
    r_out[o + (long)(n + 1) * W] = (float)r.im;
}

// ------------------------------------------------------------------ gather onto gamma (projector)
// Q(i, col0+b) = -(u(m_i, q_i)) with u = u_main (+ du, the FP32 correction of a refined solve).
template <class T>
__global__ void gather_q_kernel(const T* __restrict__ u, const float* __restrict__ du, Fold f, Band bd,
                                const int* __restrict__ gm, const int* __restrict__ gq, int ng,
                                double* __restrict__ Q, int ldq, int col0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= ng) return;
    const int m = gm[i], q = gq[i];
    C64 v = unfold_c(u, f, bd, b, m, q);
    if (du) v = cadd(v, unfold_c(du, f, bd, b, m, q));
    double* o = Q + 2 * ((long)(col0 + b) * ldq + i);
    o[0] = -v.re;
    o[1] = -v.im;
}

// ------------------------------------------------------------------ unfold to grids
// out_b(m, q) = w_b(m, q) + alpha * u_b(m, q) on the rows out_r0 + blockIdx.y (inside the
// buffer's band bd; w optional; complex interleaved FP64)
template <class T>
__device__ inline void unfold_body(const T* __restrict__ u, const float* __restrict__ du, const Fold& f, Band bd,
                                   double alpha, const double* w, long w_stride, double* out, long out_stride,
                                   const long* __restrict__ boff, int m, int q, int b) {
    const int n = f.n;
    const long node = (long)m * (n + 1) + q;
    C64 v = unfold_c(u, f, bd, b, m, q);
    if (du) v = cadd(v, unfold_c(du, f, bd, b, m, q));
    double re = alpha * v.re, im = alpha * v.im;
    if (w) {
        const double* wp = w + 2 * ((boff ? boff[b] : (long)b * w_stride) + node);
        re += wp[0];
        im += wp[1];
    }
    double* o = out + 2 * ((boff ? boff[b] : (long)b * out_stride) + node);
    o[0] = re;
    o[1] = im;
}

template <class T>
__global__ void unfold_grid_kernel(const T* __restrict__ u, const float* __restrict__ du, Fold f, Band bd,
                                   int out_r0, double alpha, const double* w, long w_stride, double* out,
                                   long out_stride, const long* __restrict__ boff) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > f.n) return;
    unfold_body<T>(u, du, f, bd, alpha, w, w_stride, out, out_stride, boff, out_r0 + blockIdx.y, q, blockIdx.z);
}

// ------------------------------------------------------------------ density on gamma for reconstruction
// w_b(gamma_i) = sum_col E(i, col) c_b(col)  (E real, c complex); w is pre-zeroed elsewhere.
__device__ inline void extend_density_body(const double* __restrict__ E, int ng, int ncol,
                                           const double* __restrict__ c, const int* __restrict__ cidx,
                                           const int* __restrict__ gm, const int* __restrict__ gq,
                                           const int* __restrict__ gside, int n, double* w, long w_stride,
                                           const long* __restrict__ woff, int i, int b) {
    // row i of E is nonzero only in its side's Dirichlet and Neumann columns
    const int M = ncol / 8, s = gside[i];
    double re = 0.0, im = 0.0;
    const double* cb = c + 2 * (long)(cidx ? cidx[b] : b) * ncol;
    for (int kind = 0; kind < 2; ++kind) {
        const int col0 = kind * 4 * M + s * M;
#pragma unroll 8
        for (int j = 0; j < M; ++j) {
            const double e = E[(long)(col0 + j) * ng + i];
            re += e * cb[2 * (col0 + j)];
            im += e * cb[2 * (col0 + j) + 1];
        }
    }
    double* o = w + 2 * ((woff ? woff[b] : (long)b * w_stride) + (long)gm[i] * (n + 1) + gq[i]);
    o[0] = re;
    o[1] = im;
}

__global__ void extend_density_kernel(const double* __restrict__ E, int ng, int ncol, const double* __restrict__ c,
                                      const int* __restrict__ cidx, const int* __restrict__ gm,
                                      const int* __restrict__ gq, const int* __restrict__ gside, int n, double* w,
                                      long w_stride, const long* __restrict__ woff) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    extend_density_body(E, ng, ncol, c, cidx, gm, gq, gside, n, w, w_stride, woff, i, blockIdx.y);
}

// Inhomogeneous part of the extension (eqs. general_extension, cart_ext_2-4, extension_split):
// at gamma node i of entry b, rho^2/2 f + rho^3/6 df/dn + rho^4/24 (d2f/dn2 - d2f/dtau2 - k^2 f)
// from the entry's jet (f, df/dn, d2f/dn2 - d2f/dtau2 at the node's foot point).
__global__ void source_extension_kernel(const double* __restrict__ rho, const int* __restrict__ gm,
                                        const int* __restrict__ gq, int ng, int n, double k,
                                        const double* const* __restrict__ jet, double* w,
                                        const long* __restrict__ woff, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    const double* J = jet[b];
    if (i >= ng || !J) return;
    const double r = rho[i], r2 = r * r;
    const double f0r = J[2 * i], f0i = J[2 * i + 1];
    const double fnr = J[2 * (ng + i)], fni = J[2 * (ng + i) + 1];
    const double ftr = J[2 * (2 * ng + i)], fti = J[2 * (2 * ng + i) + 1];
    const double a = 0.5 * r2, bb = r2 * r / 6.0, c = r2 * r2 / 24.0;
    const double vr = a * f0r + bb * fnr + c * (ftr - k * k * f0r);
    const double vi = a * f0i + bb * fni + c * (fti - k * k * f0i);
    double* o = w + 2 * (woff[b] + (long)gm[i] * (n + 1) + gq[i]);
    if (accumulate) {
        o[0] += vr;
        o[1] += vi;
    } else {
        o[0] = vr;
        o[1] = vi;
    }
}

// F[foff[b] + i] += u_b(gamma_i): the trace of an AP solution added to a right-hand side
template <class T>
__global__ void gather_add_kernel(const T* __restrict__ u, Fold f, Band bd, const int* __restrict__ gm,
                                  const int* __restrict__ gq, int ng, double* F, const long* __restrict__ foff) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= ng) return;
    const C64 v = unfold_c(u, f, bd, b, gm[i], gq[i]);
    double* o = F + 2 * (foff[b] + i);
    o[0] += v.re;
    o[1] += v.im;
}

// Extension matrix E = Ex Psi (Sec. 3.2.3-3.2.4, eqs. general_extension,
// cartesian_extension, Psi_def): column-major |gamma| x 8M*, zero outside the
// node's side.  For gamma node i on side s, at signed distance rho from the
// side line and side parameter t, with psi = T_j(t) and tangential derivatives
// psi^(p) = (2 / side length)^p T_j^(p)(t):
//   Dirichlet column s M* + j:       psi + rho^2/2 (-psi_tt - k^2 psi)
//                                    + rho^4/24 (psi_tttt + 2 k^2 psi_tt + k^4 psi)
//   Neumann column 4M* + s M* + j:   rho psi + rho^3/6 (-psi_tt - k^2 psi)
// (the Taylor expansion in rho of a Helmholtz solution with u = psi, du/dn = 0
// resp. u = 0, du/dn = psi on the side, normal derivatives replaced through the
// equation).  T_j^(p) by the differentiated recurrence
// T_{j+1}^(p) = 2 t T_j^(p) + 2 p T_j^(p-1) - T_{j-1}^(p), one thread per node.
// extension_row writes the 2M* entries of the node's side; extension_kernel leaves the
// other 6M* entries of the row as they are (the caller zeroes E), geom_setup_kernel
// writes them as zeros.
__device__ inline void extension_row(int s, double t, double r, double slen, int ng, double k, int M,
                                     double* __restrict__ E, int deriv, int i) {
    const double sc = 2.0 / slen, sc2 = sc * sc, sc4 = sc2 * sc2;
    const double k2 = k * k, k4 = k2 * k2;
    const double r2 = r * r, r3 = r2 * r, r4 = r2 * r2;
    double cur[5] = {1.0, 0.0, 0.0, 0.0, 0.0};    // T_j^(p), p = 0..4
    double prev[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // T_{j-1}^(p)
    for (int j = 0; j < M; ++j) {
        const double p0 = cur[0], p2 = sc2 * cur[2], p4 = sc4 * cur[4];
        if (deriv) {   // d/d(k^2): -rho^2/2 psi + rho^4/24 (2 psi'' + 2 k^2 psi) and -rho^3/6 psi
            E[(long)(s * M + j) * ng + i] = -0.5 * r2 * p0 + (r4 / 24.0) * (2.0 * p2 + 2.0 * k2 * p0);
            E[(long)(4 * M + s * M + j) * ng + i] = -(r3 / 6.0) * p0;
        } else {
            E[(long)(s * M + j) * ng + i] =
                p0 + 0.5 * r2 * (-p2 - k2 * p0) + (r4 / 24.0) * (p4 + 2.0 * k2 * p2 + k4 * p0);
            E[(long)(4 * M + s * M + j) * ng + i] = r * p0 + (r3 / 6.0) * (-p2 - k2 * p0);
        }
        double nxt[5];
        if (j == 0) {
            nxt[0] = t;
            nxt[1] = 1.0;
            nxt[2] = nxt[3] = nxt[4] = 0.0;
        } else {
#pragma unroll
            for (int p = 0; p < 5; ++p) nxt[p] = 2.0 * t * cur[p] - prev[p] + (p ? 2.0 * p * cur[p - 1] : 0.0);
        }
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            prev[p] = cur[p];
            cur[p] = nxt[p];
        }
    }
}

__global__ void extension_kernel(const int* __restrict__ side, const double* __restrict__ rho,
                                 const double* __restrict__ tpar, const double* __restrict__ slen, int ng, double k,
                                 int M, double* __restrict__ E, int deriv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    extension_row(side[i], tpar[i], rho[i], slen[i], ng, k, M, E, deriv, i);
}

// The set-up of one build in one launch (entry blockIdx.y; the x workgroups stride over
// the entry's work): for a geometry new to the context, its gamma node tables copied
// from the call's upload into its own buffer and its node -> gamma map filled with -1;
// for a projector, the full rows of E (zero outside the node's side).
__global__ void __launch_bounds__(256) geom_setup_kernel(const GeomJob* __restrict__ jobs) {
    const GeomJob jb = jobs[blockIdx.y];
    const long stride = (long)gridDim.x * blockDim.x;
    const long t0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned* src = reinterpret_cast<const unsigned*>(jb.src);
    unsigned* dst = reinterpret_cast<unsigned*>(jb.meta);
    for (long w = t0; w < jb.meta_words; w += stride) dst[w] = src[w];
    const int M = jb.M, ng = jb.E ? jb.ng : 0;
    for (long i = t0; i < ng; i += stride) {
        const int s = jb.side[i];
        for (int kind = 0; kind < 2; ++kind)
            for (int q = 0; q < 4; ++q) {
                if (q == s) continue;
                double* col = jb.E + (long)(kind * 4 * M + q * M) * ng + i;
                for (int j = 0; j < M; ++j) col[(long)j * ng] = 0.0;
            }
        extension_row(s, jb.t[i], jb.rho[i], jb.slen[i], ng, jb.k, M, jb.E, 0, (int)i);
    }
    if (!jb.gidx) return;
    const long nodes = (long)(jb.n + 1) * (jb.n + 1);
    for (long v = t0; v < nodes; v += stride) jb.gidx[v] = -1;
}

// gidx[gm[i] (n+1) + gq[i]] = i for every entry with a node map (after geom_setup_kernel)
__global__ void __launch_bounds__(256) gamma_index_jobs_kernel(const GeomJob* __restrict__ jobs) {
    const GeomJob jb = jobs[blockIdx.y];
    if (!jb.gidx) return;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < jb.ng; i += (long)gridDim.x * blockDim.x)
        jb.gidx[jb.gm[i] * (jb.n + 1) + jb.gq[i]] = (int)i;
}

inline unsigned grid_for(long total, int block = 256) {
    long g = (total + block - 1) / block;
    if (g > 1 << 20) g = 1 << 20;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

static void check_batch(int R) {
    if (R > 65535) throw Error(MDP_ERR_ARG, "batch too large for one launch");
}

static void check_band(const Band& bd, int n) {
    if (bd.r0 < 0 || bd.nr < 1 || bd.r0 + bd.nr > n + 1) throw Error(MDP_ERR_ARG, "row band outside the grid");
}

template <class T>
void launch_fold_rhs(const SrcDesc& s, int n, const Fold& f, StencilCoef sc, int R, bool cplx, Band bd, T* out,
                     hipStream_t st) {
    check_batch(R);
    check_band(bd, n);
    SrcEval ev{s, n, sc};
    const int bx = f.W < 256 ? f.W : 256;
    dim3 grid((f.W + bx - 1) / bx, bd.nr, R);
    hipLaunchKernelGGL(fold_rhs_kernel<T>, grid, dim3(bx), 0, st, ev, f, cplx ? 2 : 1, bd, out);
    MDP_HIP(hipGetLastError());
}

template <class T>
void launch_tridiag(const T* in, int planes_in, T* out, const T* fac, const T* colc, int n, const Fold& f, int R,
                    Band bd, hipStream_t st) {
    check_batch(R);
    check_band(bd, n);
    // one column per thread while that gives a few thousand wavefronts; otherwise up to 16
    // row segments of at least 8 rows per column
    const long waves = (long)R * ((f.W + 63) / 64);
    int P = (int)std::min<long>(16, (4096 + waves - 1) / waves);
    P = std::min(P, (bd.nr + 7) / 8);
    if (P <= 1) {
        dim3 grid((f.W + 255) / 256, R);
        hipLaunchKernelGGL(tridiag_kernel<T>, grid, dim3(256), 0, st, in, planes_in, out, fac, colc, n, f.W, R, bd);
    } else {
        const int Lseg = (bd.nr + P - 1) / P;
        P = (bd.nr + Lseg - 1) / Lseg;
        dim3 grid((f.W + 63) / 64, R);
        hipLaunchKernelGGL(tridiag_part_kernel<T>, grid, dim3(64 * P), 0, st, in, planes_in, out, fac, colc, n, f.W,
                           bd, P, Lseg);
    }
    MDP_HIP(hipGetLastError());
}

void launch_residual(const SrcDesc& s, int n, const Fold& f, StencilCoef sc, EndRowCoef ec, int R, bool,
                     const float* u32, float* r_out, hipStream_t st) {
    check_batch(R);
    SrcEval ev{s, n, sc};
    const int bx = f.W < 256 ? f.W : 256;
    dim3 grid((f.W + bx - 1) / bx, n + 1, R);
    hipLaunchKernelGGL(residual_kernel, grid, dim3(bx), 0, st, ev, ec, f, u32, r_out);
    MDP_HIP(hipGetLastError());
}

template <class T>
void launch_gather_q(const T* u, const float* du, int n, const Fold& f, Band bd, const int* gm, const int* gq, int ng,
                     int R, double* Q, int ldq, int col0, hipStream_t st) {
    check_batch(R);
    check_band(bd, n);
    dim3 grid((ng + 255) / 256, R);
    hipLaunchKernelGGL(gather_q_kernel<T>, grid, dim3(256), 0, st, u, du, f, bd, gm, gq, ng, Q, ldq, col0);
    MDP_HIP(hipGetLastError());
}

template <class T>
void launch_unfold_grid(const T* u, const float* du, int n, const Fold& f, Band bd, Band rows, int R, const double* w,
                        long w_stride, double* out, long out_stride, const long* boff, hipStream_t st) {
    check_batch(R);
    check_band(bd, n);
    if (rows.r0 < bd.r0 || rows.nr < 1 || rows.r0 + rows.nr > bd.r0 + bd.nr)
        throw Error(MDP_ERR_ARG, "output rows outside the solved band");
    double alpha = w ? -1.0 : 1.0;
    dim3 grid((n + 1 + 255) / 256, rows.nr, R);
    hipLaunchKernelGGL(unfold_grid_kernel<T>, grid, dim3(256), 0, st, u, du, f, bd, rows.r0, alpha, w, w_stride, out,
                       out_stride, boff);
    MDP_HIP(hipGetLastError());
}

void launch_source_extension(const double* rho, const int* gm, const int* gq, int ng, int n, double k,
                             const double* const* jet, int R, double* w, const long* woff, bool accumulate,
                             hipStream_t st) {
    check_batch(R);
    if (ng <= 0 || R <= 0) return;
    dim3 grid((ng + 255) / 256, R);
    hipLaunchKernelGGL(source_extension_kernel, grid, dim3(256), 0, st, rho, gm, gq, ng, n, k, jet, w, woff,
                       accumulate ? 1 : 0);
    MDP_HIP(hipGetLastError());
}

template <class T>
void launch_gather_add(const T* u, int n, const Fold& f, Band bd, const int* gm, const int* gq, int ng, int R,
                       double* F, const long* foff, hipStream_t st) {
    check_batch(R);
    check_band(bd, n);
    if (ng <= 0 || R <= 0) return;
    dim3 grid((ng + 255) / 256, R);
    hipLaunchKernelGGL(gather_add_kernel<T>, grid, dim3(256), 0, st, u, f, bd, gm, gq, ng, F, foff);
    MDP_HIP(hipGetLastError());
}
template void launch_gather_add<double>(const double*, int, const Fold&, Band, const int*, const int*, int, int,
                                        double*, const long*, hipStream_t);
template void launch_gather_add<float>(const float*, int, const Fold&, Band, const int*, const int*, int, int,
                                       double*, const long*, hipStream_t);

void launch_extend_density(const double* E, int ng, int ncol, const double* c, const int* cidx, int R, const int* gm,
                           const int* gq, const int* gside, int n, double* w, long w_stride, const long* woff,
                           hipStream_t st) {
    check_batch(R);
    if (ncol % 8) throw Error(MDP_ERR_ARG, "extension matrix width must be 8 M*");
    dim3 grid((ng + 255) / 256, R);
    hipLaunchKernelGGL(extend_density_kernel, grid, dim3(256), 0, st, E, ng, ncol, c, cidx, gm, gq, gside, n, w,
                       w_stride, woff);
    MDP_HIP(hipGetLastError());
}

template void launch_fold_rhs<double>(const SrcDesc&, int, const Fold&, StencilCoef, int, bool, Band, double*,
                                      hipStream_t);
template void launch_fold_rhs<float>(const SrcDesc&, int, const Fold&, StencilCoef, int, bool, Band, float*,
                                     hipStream_t);
template void launch_tridiag<double>(const double*, int, double*, const double*, const double*, int, const Fold&, int,
                                     Band, hipStream_t);
template void launch_tridiag<float>(const float*, int, float*, const float*, const float*, int, const Fold&, int,
                                    Band, hipStream_t);
template void launch_gather_q<double>(const double*, const float*, int, const Fold&, Band, const int*, const int*, int,
                                      int, double*, int, int, hipStream_t);
template void launch_gather_q<float>(const float*, const float*, int, const Fold&, Band, const int*, const int*, int,
                                     int, double*, int, int, hipStream_t);
template void launch_unfold_grid<double>(const double*, const float*, int, const Fold&, Band, Band, int,
                                         const double*, long, double*, long, const long*, hipStream_t);
template void launch_unfold_grid<float>(const float*, const float*, int, const Fold&, Band, Band, int, const double*,
                                        long, double*, long, const long*, hipStream_t);


// ============================================================================
// Projector build, support-in / gamma-out form (FP64).
//
// For a projector column the right-hand side g = L^(h) w |_{M+} (w on gamma)
// lives on the two outermost rings of the M+ box [m_lo, m_hi] x [q_lo, q_hi],
// and Q needs the solution only on gamma.  With the box symmetric in y
// (q_hi = n - q_lo):
//   * rows m_lo, m_lo+1, m_hi-1, m_hi ("special input rows") are dense in q:
//     their folded rows go through the MFMA sine GEMM (4 rows per RHS);
//   * every other row has g only at q_lo, q_lo+1, q_hi-1, q_hi, i.e. two
//     entries per folded block: its transform is two multiply-adds per mode,
//     done on the fly inside the tridiagonal sweep;
//   * on gamma, rows m_lo-1, m_lo, m_hi, m_hi+1 are full: the sweep writes
//     their mode-space values to a compact buffer for a small inverse GEMM;
//     every other gamma row needs u only at q_lo-1, q_lo and their mirrors,
//     i.e. the folded synthesis values A, B at q_lo-1 and q_lo, which are sums
//     over the modes: reduced across the wavefront as the sweep produces them.
// The tridiagonal sweep keeps nothing of the column in HBM: the forward pass
// stores y only at the end of every K-row segment, and the backward pass
// recomputes each segment's y in registers before walking back through it.
// ============================================================================
namespace {

struct RingGeom {
    int m_lo, m_hi, q_lo, q_hi;
};

__device__ inline int special_in(const RingGeom& r, int m) {
    if (m == r.m_lo) return 0;
    if (m == r.m_lo + 1) return 1;
    if (m == r.m_hi - 1) return 2;
    if (m == r.m_hi) return 3;
    return -1;
}
__device__ inline int special_out(const RingGeom& r, int m) {
    if (m == r.m_lo - 1) return 0;
    if (m == r.m_lo) return 1;
    if (m == r.m_hi) return 2;
    if (m == r.m_hi + 1) return 3;
    return -1;
}

// gc[b][m][4] = (g_lo + g_hi, g_lo1 + g_hi1, g_lo - g_hi, g_lo1 - g_hi1) for
// every row m = 0..n, with g_lo = g(m, q_lo), g_lo1 = g(m, q_lo+1),
// g_hi1 = g(m, q_hi-1), g_hi = g(m, q_hi): the folded ring entries of a
// non-special box row (zero on the special rows and outside the box);
// spec[b][s][W] = folded special input row s.
// Work item t of RHS b: t <= n a gc row, otherwise one folded special entry.
// The job of global column b (jobs sorted by b0; uniform over the workgroup).
__device__ inline int find_job(const FusedJob* __restrict__ jobs, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One workgroup per column.  The column's density w = E(:, col) (nonzero on gamma only)
// is spread once into LDS: the full rows m_lo-1 .. m_lo+2 and m_hi-2 .. m_hi+1 (D: the
// neighbourhoods of the special rows) and, for every row, its values at q_lo-1, q_lo,
// q_hi, q_hi+1 (S: on the other rows gamma holds only those four nodes), from the
// gamma lists (coalesced reads of E, gm, gq).  The stencil L^(h) w at an M+ node then
// reads its nine taps from LDS, in the same order as the general right-hand side.
// LDS: 12 (n+1) doubles.
template <class T>
__global__ void __launch_bounds__(256)
fold_ring_kernel(const FusedJob* __restrict__ jobs, int njobs) {
    extern __shared__ double lds_fr[];
    const int gcol = blockIdx.x;
    const FusedJob& J = jobs[find_job(jobs, njobs, gcol)];
    const Fold f = J.f;
    const RingGeom rg{J.src.m_lo, J.src.m_hi, J.src.q_lo, J.src.q_hi};
    T* __restrict__ gc = reinterpret_cast<T*>(J.gc);
    T* __restrict__ spec = reinterpret_cast<T*>(J.spec);
    const int n = f.n, n1 = n + 1, p = f.p, W = f.W, b = gcol - J.b0;
    const int m_lo = rg.m_lo, m_hi = rg.m_hi, q_lo = rg.q_lo, q_hi = rg.q_hi;
    double* D = lds_fr;          // [8][n+1]
    double* S = D + 8 * n1;      // [n+1][4]
    for (int e = threadIdx.x; e < 12 * n1; e += 256) lds_fr[e] = 0.0;
    __syncthreads();
    const double* __restrict__ w = J.src.E + (long)(J.src.col0 + b) * J.src.ldE;
    const int* __restrict__ gm = J.gm;
    const int* __restrict__ gq = J.gq;
    auto strip_col = [&](int q) { return (q == q_lo - 1) ? 0 : (q == q_lo) ? 1 : (q == q_hi) ? 2 : (q == q_hi + 1) ? 3 : -1; };
    for (int i = threadIdx.x; i < J.ng; i += 256) {
        const int m = gm[i], q = gq[i];
        const double v = w[i];
        const int r0 = m - (m_lo - 1), r1 = m - (m_hi - 2);
        if (r0 >= 0 && r0 < 4) D[r0 * n1 + q] = v;
        if (r1 >= 0 && r1 < 4) D[(4 + r1) * n1 + q] = v;
        const int k = strip_col(q);
        if (k >= 0) S[m * 4 + k] = v;
    }
    __syncthreads();
    auto wv = [&](int m, int q) -> double {
        const int r0 = m - (m_lo - 1), r1 = m - (m_hi - 2);
        if (r0 >= 0 && r0 < 4) return D[r0 * n1 + q];
        if (r1 >= 0 && r1 < 4) return D[(4 + r1) * n1 + q];
        const int k = strip_col(q);
        return k >= 0 ? S[m * 4 + k] : 0.0;
    };
    const StencilCoef sc = J.sc;
    // L^(h) w at node (m, q), zero off M+ (eq. FD_scheme restricted to M+)
    auto rhs = [&](int m, int q) -> double {
        if (m < m_lo || m > m_hi || q < q_lo || q > q_hi) return 0.0;
        const double ce = wv(m + 1, q) + wv(m - 1, q) + wv(m, q + 1) + wv(m, q - 1);
        const double cc = wv(m + 1, q + 1) + wv(m - 1, q + 1) + wv(m + 1, q - 1) + wv(m - 1, q - 1);
        return sc.c0 * wv(m, q) + sc.ce * ce + sc.cc * cc;
    };
    // ring table of the swept rows m_lo-1 .. m_hi+1 (zero on the special rows and outside the box)
    for (int m = m_lo - 1 + (int)threadIdx.x; m <= m_hi + 1; m += 256) {
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
        if (m >= m_lo && m <= m_hi && special_in(rg, m) < 0) {
            v0 = rhs(m, q_lo);
            v1 = rhs(m, q_lo + 1);
            v2 = rhs(m, q_hi - 1);
            v3 = rhs(m, q_hi);
        }
        T* o = gc + ((long)b * n1 + m) * 4;
        o[0] = (T)(v0 + v3);
        o[1] = (T)(v1 + v2);
        o[2] = (T)(v0 - v3);
        o[3] = (T)(v1 - v2);
    }
    // folded special input rows: the stencil of special row s reads rows m-1..m+1, all held
    // full in D (rows m_lo-1..m_lo+2 for s = 0, 1 and m_hi-2..m_hi+1 for s = 2, 3); each pair
    // of mirrored nodes (q, n - q) is evaluated once for its odd-mode column q - 1 (the sum)
    // and its even-mode column P1 + q - 1 (the difference)
    const int P1 = f.P1;
    for (int i = threadIdx.x; i < 4 * P1; i += 256) {
        const int s_ = i / P1, j = i - s_ * P1, q = j + 1;
        const int m = (s_ == 0) ? m_lo : (s_ == 1) ? m_lo + 1 : (s_ == 2) ? m_hi - 1 : m_hi;
        const double* Dm = D + ((s_ < 2 ? m - (m_lo - 1) : 4 + m - (m_hi - 2)) * n1);   // row m of D
        auto rhs_d = [&](int qq) -> double {   // rhs(m, qq) from D alone
            if (qq < q_lo || qq > q_hi) return 0.0;
            const double ce = Dm[n1 + qq] + Dm[-n1 + qq] + Dm[qq + 1] + Dm[qq - 1];
            const double cc = Dm[n1 + qq + 1] + Dm[-n1 + qq + 1] + Dm[n1 + qq - 1] + Dm[-n1 + qq - 1];
            return sc.c0 * Dm[qq] + sc.ce * ce + sc.cc * cc;
        };
        double ve = 0.0, vo = 0.0;
        if (q < p) {
            const double r1 = rhs_d(q), r2 = rhs_d(n - q);
            vo = r1 + r2;
            ve = r1 - r2;
        } else if (q == p) {
            vo = rhs_d(p);
        }
        T* o = spec + ((long)b * 4 + s_) * W;
        o[j] = (T)vo;
        if (P1 + j < W) o[P1 + j] = (T)ve;
    }
}

// Q(i, col0+b) = -u(m_i, q_i): the full gamma rows from the synthesis rows us
// ([b][plane][4][W], output of the inverse sine GEMM of xs), the others from
// the thin partial sums (odd-mode blocks give A, even-mode blocks B; with pair_blocks the
// sweep summed each pair of 64-column blocks 2k, 2k + 1 not straddling P1 into slot 2k).
// One workgroup per column (one job lookup), its threads over the column's gamma nodes.
template <class T>
__global__ void __launch_bounds__(256) gather_q_fused_kernel(const FusedJob* __restrict__ jobs, int njobs,
                                                             int pair_blocks) {
    const int gcol = blockIdx.x;
    const FusedJob& J = jobs[find_job(jobs, njobs, gcol)];
    const int b = gcol - J.b0;
    const Fold f = J.f;
    const RingGeom rg{J.src.m_lo, J.src.m_hi, J.src.q_lo, J.src.q_hi};
    const T* __restrict__ us = reinterpret_cast<const T*>(J.us);
    const T* __restrict__ thin = reinterpret_cast<const T*>(J.thin);
    const int* __restrict__ gm = J.gm;
    const int* __restrict__ gq = J.gq;
    const int rows_pad = J.rows_pad, ldq = J.ldq, col0 = J.src.col0;
    double* __restrict__ Q = J.Q;
    const int n = f.n, p = f.p, W = f.W;
    for (int i = threadIdx.x; i < J.ng; i += blockDim.x) {
    const int m = gm[i], q = gq[i];
    double vre, vim;
    const int so = special_out(rg, m);
    if (so >= 0) {
        double v[2];
        for (int pl = 0; pl < 2; ++pl) {
            const T* row = us + (((long)b * 2 + pl) * 4 + so) * W;
            double u;
            if (q <= 0 || q >= n) u = 0.0;
            else if (q == p) u = (double)row[p - 1];
            else if (q < p) u = (double)row[q - 1] + (double)row[f.P1 + q - 1];
            else u = (double)row[n - q - 1] - (double)row[f.P1 + n - q - 1];
            v[pl] = u;
        }
        vre = v[0];
        vim = v[1];
    } else {
        const int qq = (q <= p) ? q : n - q;
        const double sgn = (q <= p) ? 1.0 : -1.0;
        const int k2 = (qq == rg.q_lo - 1) ? 0 : 2;
        const int nb = W / 64, nb1 = f.P1 / 64;
        double A0 = 0.0, A1 = 0.0, B0 = 0.0, B1 = 0.0;
        for (int w = 0; w < nb; ++w) {
            if (pair_blocks && (w & 1) && w * 64 != f.P1) continue;   // summed into slot w - 1
            const T* t = thin + (((long)b * nb + w) * rows_pad + (m - rg.m_lo + 1)) * 4 + k2;
            if (w < nb1) { A0 += (double)t[0]; A1 += (double)t[1]; }
            else { B0 += (double)t[0]; B1 += (double)t[1]; }
        }
        vre = A0 + sgn * B0;
        vim = A1 + sgn * B1;
    }
    double* o = Q + 2 * ((long)(col0 + b) * ldq + i);
    o[0] = -vre;
    o[1] = -vim;
    }
}

// ------------------------------------------------------------------ batched solves across plans
__device__ inline int find_solve_job(const SolveJob* __restrict__ jobs, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void extend_density_jobs_kernel(const SolveJob* __restrict__ jobs, int njobs, double* grids,
                                           const double* __restrict__ c) {
    const SolveJob& J = jobs[find_solve_job(jobs, njobs, blockIdx.y)];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= J.ng) return;
    extend_density_body(J.E, J.ng, J.ncol, c, J.cidx, J.gm, J.gq, J.gside, J.f.n, grids, 0, J.src.goff, i,
                        blockIdx.y - J.b0);
}

// rows kJobRows blockIdx.x .. of entry blockIdx.y per workgroup (one job lookup), the
// threads over the row's columns
constexpr int kJobRows = 8;

__global__ void __launch_bounds__(256)
fold_rhs_jobs_kernel(const SolveJob* __restrict__ jobs, int njobs) {
    const SolveJob& J = jobs[find_solve_job(jobs, njobs, blockIdx.y)];
    const SrcEval ev{J.src, J.f.n, J.sc};
    const int r1 = min(J.bd.nr, (int)(blockIdx.x + 1) * kJobRows);
    for (int r = blockIdx.x * kJobRows; r < r1; ++r)
        for (int j = threadIdx.x; j < J.f.P1; j += blockDim.x)
            fold_rhs_pair_body<double>(ev, J.f, 2, J.bd, J.A, j, J.bd.r0 + r, blockIdx.y - J.b0);
}

__global__ void __launch_bounds__(256)
tridiag_jobs_kernel(const SolveJob* __restrict__ jobs, int njobs) {
    const SolveJob& J = jobs[find_solve_job(jobs, njobs, blockIdx.y)];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= J.f.W) return;
    if (J.adjoint) tridiag_adj_body(J.B, 2, J.A, J.fac, J.colc, J.f.n, J.f.W, c, blockIdx.y - J.b0);
    else tridiag_body<double>(J.B, 2, J.A, J.fac, J.colc, J.f.n, J.f.W, J.bd, c, blockIdx.y - J.b0);
}

__global__ void __launch_bounds__(256) unfold_jobs_kernel(const SolveJob* __restrict__ jobs, int njobs,
                                                          double* grids) {
    const SolveJob& J = jobs[find_solve_job(jobs, njobs, blockIdx.y)];
    const int r1 = min(J.bd.nr, (int)(blockIdx.x + 1) * kJobRows), b = blockIdx.y - J.b0;
    for (int r = blockIdx.x * kJobRows; r < r1; ++r)
        for (int q = threadIdx.x; q <= J.f.n; q += blockDim.x) {
            if (J.out)   // the solution itself into separate grids
                unfold_body<double>(J.B, nullptr, J.f, J.bd, 1.0, nullptr, 0, J.out, 0, J.ooff, J.bd.r0 + r, q, b);
            else         // w - u in place
                unfold_body<double>(J.B, nullptr, J.f, J.bd, -1.0, grids, 0, grids, 0, J.src.goff, J.bd.r0 + r, q, b);
        }
}

}  // namespace

void launch_extension(const int* side, const double* rho, const double* t, const double* slen, int ng, double k,
                      int m_star, double* E, hipStream_t st, int deriv) {
    if (ng <= 0) return;
    hipLaunchKernelGGL(extension_kernel, dim3((ng + 255) / 256), dim3(256), 0, st, side, rho, t, slen, ng, k, m_star,
                       E, deriv);
    MDP_HIP(hipGetLastError());
}

void launch_geom_setup(const GeomJob* jobs_dev, int count, int max_nodes, hipStream_t st) {
    if (count <= 0) return;
    if (count > 65535) throw Error(MDP_ERR_ARG, "too many projectors for one set-up launch");
    const unsigned gx = (unsigned)std::max(1, std::min(64, (max_nodes + 255) / 256));
    hipLaunchKernelGGL(geom_setup_kernel, dim3(gx, count), dim3(256), 0, st, jobs_dev);
    MDP_HIP(hipGetLastError());
    hipLaunchKernelGGL(gamma_index_jobs_kernel, dim3(std::min(gx, 16u), count), dim3(256), 0, st, jobs_dev);
    MDP_HIP(hipGetLastError());
}

bool fused_projector_supported(const Fold& f, int m_lo, int m_hi, int q_lo, int q_hi) {
    return q_hi == f.n - q_lo && q_lo >= 2 && q_lo <= f.p - 2 && m_lo >= 2 && m_hi <= f.n - 2 && m_hi - m_lo >= 3 &&
           f.W % 64 == 0 && f.P1 % 64 == 0 && fold_ring_lds_bytes(f.n) <= kFoldRingMaxLds;
}

int fused_segments(int m_lo, int m_hi) { return (m_hi - m_lo + 3 + FUSED_K - 1) / FUSED_K; }

void launch_extend_density_jobs(const SolveJob* jobs, int njobs, int total, int max_ng, double* grids,
                                const double* c, hipStream_t st) {
    if (njobs <= 0 || total <= 0 || max_ng <= 0) return;
    check_batch(total);
    hipLaunchKernelGGL(extend_density_jobs_kernel, dim3((max_ng + 255) / 256, total), dim3(256), 0, st, jobs, njobs,
                       grids, c);
    MDP_HIP(hipGetLastError());
}

void launch_fold_rhs_jobs(const SolveJob* jobs, int njobs, int total, int max_w, int max_nr, hipStream_t st) {
    if (njobs <= 0 || total <= 0) return;
    check_batch(total);
    (void)max_w;
    hipLaunchKernelGGL(fold_rhs_jobs_kernel, dim3((max_nr + kJobRows - 1) / kJobRows, total), dim3(256), 0, st, jobs,
                       njobs);
    MDP_HIP(hipGetLastError());
}

void launch_tridiag_jobs(const SolveJob* jobs, int njobs, int total, int max_w, hipStream_t st) {
    if (njobs <= 0 || total <= 0) return;
    check_batch(total);
    hipLaunchKernelGGL(tridiag_jobs_kernel, dim3((max_w + 255) / 256, total), dim3(256), 0, st, jobs, njobs);
    MDP_HIP(hipGetLastError());
}

void launch_unfold_jobs(const SolveJob* jobs, int njobs, int total, int max_n, int max_nr, double* grids,
                        hipStream_t st) {
    if (njobs <= 0 || total <= 0) return;
    check_batch(total);
    (void)max_n;
    hipLaunchKernelGGL(unfold_jobs_kernel, dim3((max_nr + kJobRows - 1) / kJobRows, total), dim3(256), 0, st, jobs,
                       njobs, grids);
    MDP_HIP(hipGetLastError());
}

static dim3 flat_grid(int per_col, int total) {
    const long blocks = (long)per_col * total;
    if (blocks > 0x7fffffffL) throw Error(MDP_ERR_ARG, "too many projector columns for one launch");
    return dim3((unsigned)blocks);
}

template <class T>
void launch_fold_ring_jobs(const FusedJob* jobs, int njobs, int total, int max_n, hipStream_t st) {
    if (njobs <= 0 || total <= 0) return;
    const size_t lds = fold_ring_lds_bytes(max_n);
    if (lds > kFoldRingMaxLds) throw Error(MDP_ERR_ARG, "grid too large for the fused projector route");
    static const bool lds_set = [] {   // more than 64 KB of dynamic LDS must be allowed explicitly
        MDP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&fold_ring_kernel<T>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFoldRingMaxLds));
        return true;
    }();
    (void)lds_set;
    hipLaunchKernelGGL(fold_ring_kernel<T>, flat_grid(1, total), dim3(256), lds, st, jobs, njobs);
    MDP_HIP(hipGetLastError());
}
template void launch_fold_ring_jobs<double>(const FusedJob*, int, int, int, hipStream_t);
template void launch_fold_ring_jobs<float>(const FusedJob*, int, int, int, hipStream_t);

template <class T>
void launch_gather_q_fused_jobs(const FusedJob* jobs, int njobs, int total, int max_ng, int sweep_cols,
                                hipStream_t st) {
    if (njobs <= 0 || total <= 0) return;
    (void)max_ng;
    hipLaunchKernelGGL(gather_q_fused_kernel<T>, flat_grid(1, total), dim3(256), 0, st, jobs, njobs,
                       sweep_cols == 2 ? 1 : 0);
    MDP_HIP(hipGetLastError());
}
template void launch_gather_q_fused_jobs<double>(const FusedJob*, int, int, int, int, hipStream_t);
template void launch_gather_q_fused_jobs<float>(const FusedJob*, int, int, int, int, hipStream_t);

// ------------------------------------------------------------------ allocation-free solves
// The batch buffers of the allocation-free AP solve: a static device array, which every
// device the library runs on holds until the process ends.  In host code the array's
// name stands for a host-side shadow, not a device address: host code uses only the
// address that hipGetSymbolAddress returns for the current device (kept per device).
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;
}  // namespace

void* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));   // `device` is current
    if (e != hipSuccess || !ptr)
        throw Error(MDP_ERR_HIP, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return ptr;
}

}  // namespace mdp
