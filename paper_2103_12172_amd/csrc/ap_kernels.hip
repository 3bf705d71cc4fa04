// Memory-bound kernels of the auxiliary-problem (AP) solve and of the
// projector / reconstruction steps.
//
// Data layout in HBM (one batch of R right-hand sides, n even, p = n/2):
//   folded rows  buf[((b*planes + pl)*(n+1) + m)*W + c]
//     b = right-hand side, pl = 0 (real) / 1 (imaginary) plane, m = 0..n the
//     x index, c the folded column (block 1: e_q or odd modes, block 2: o_q or
//     even modes, see Fold).  Columns are contiguous, so a wavefront walking m
//     for 64 consecutive columns reads 64 consecutive elements per step.
//   grids        complex interleaved FP64, (n+1)^2 per function, index m*(n+1)+q.
#include <hip/hip_complex.h>

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
        const double* g = d.grid + 2 * ((long)b * d.grid_stride + (long)m * (n + 1) + q);
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
    // right-hand side g(m, q) of the AP at an interior node (zero on the end rows)
    __device__ inline C64 rhs(int b, int m, int q) const {
        if (m <= 0 || m >= n || q <= 0 || q >= n) return {0.0, 0.0};
        if (d.kind == Src::GRID) return wgrid(b, m, q);
        if (!in_mplus(m, q)) return {0.0, 0.0};
        return stencil(b, m, q);
    }
};

// ------------------------------------------------------------------ fold RHS
// out row (b, m): block 1 col c = q-1 (q = 1..p):   e_q = g_q + g_{n-q} (e_p = g_p)
//                 block 2 col c = P1+q-1 (q < p):   o_q = g_q - g_{n-q}
template <class T>
__global__ void __launch_bounds__(256)
fold_rhs_kernel(SrcEval ev, Fold f, int planes, T* __restrict__ out) {
    const int n = f.n, p = f.p, W = f.W;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y, b = blockIdx.z;
    if (c >= W) return;
    C64 v = {0.0, 0.0};
    if (c < f.P1) {
        const int q = c + 1;
        if (q < p) v = cadd(ev.rhs(b, m, q), ev.rhs(b, m, n - q));
        else if (q == p) v = ev.rhs(b, m, p);
    } else {
        const int q = c - f.P1 + 1;
        if (q < p) v = csub(ev.rhs(b, m, q), ev.rhs(b, m, n - q));
    }
    const long o = (((long)b * planes) * (n + 1) + m) * W + c;
    out[o] = (T)v.re;
    if (planes == 2) out[o + (long)(n + 1) * W] = (T)v.im;
}

// ------------------------------------------------------------------ tridiagonal solve per mode
// For column c (one sine mode) and right-hand side b: rows m = 0..n,
//   Thomas with precomputed factors: y_0 = f_0, y_m = f_m - l_m y_{m-1};
//   x_n = r_n y_n, x_m = r_m (y_m - s_m x_{m+1}) with s_0 = sup0 (complex end
//   row), s_m = a_c (interior off-diagonal) otherwise.
// fac planes: [0] l.re [1] l.im [2] r.re [3] r.im, each (n+1) x W; colc: [0] a, [1] sup0.re, [2] sup0.im.
// y is kept in `out` between the sweeps.
template <class T>
__global__ void __launch_bounds__(256)
tridiag_kernel(const T* __restrict__ in, int planes_in, T* __restrict__ out, const T* __restrict__ fac,
               const T* __restrict__ colc, int n, int W, int R) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= W || b >= R) return;
    const long plane = (long)(n + 1) * W;
    const T* fin_re = in + (long)b * planes_in * plane + c;
    const T* fin_im = (planes_in == 2) ? fin_re + plane : nullptr;
    T* o_re = out + (long)b * 2 * plane + c;
    T* o_im = o_re + plane;
    const T* l_re = fac + c;
    const T* l_im = fac + plane + c;
    const T* r_re = fac + 2 * plane + c;
    const T* r_im = fac + 3 * plane + c;
    const T a = colc[c], s0r = colc[W + c], s0i = colc[2 * W + c];

    // forward sweep
    T yr = fin_re[0], yi = fin_im ? fin_im[0] : T(0);
    o_re[0] = yr;
    o_im[0] = yi;
    constexpr int U = 4;
    int m = 1;
    for (; m + U - 1 <= n; m += U) {
        T fr[U], fi[U], lr[U], li[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            long off = (long)(m + u) * W;
            fr[u] = fin_re[off];
            fi[u] = fin_im ? fin_im[off] : T(0);
            lr[u] = l_re[off];
            li[u] = l_im[off];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            T nr = fr[u] - (lr[u] * yr - li[u] * yi);
            T ni = fi[u] - (lr[u] * yi + li[u] * yr);
            yr = nr;
            yi = ni;
            long off = (long)(m + u) * W;
            o_re[off] = yr;
            o_im[off] = yi;
        }
    }
    for (; m <= n; ++m) {
        long off = (long)m * W;
        T fr = fin_re[off], fi = fin_im ? fin_im[off] : T(0);
        T lr = l_re[off], li = l_im[off];
        T nr = fr - (lr * yr - li * yi);
        T ni = fi - (lr * yi + li * yr);
        yr = nr;
        yi = ni;
        o_re[off] = yr;
        o_im[off] = yi;
    }
    // backward sweep
    {
        long off = (long)n * W;
        T rr = r_re[off], ri = r_im[off];
        T xr = rr * yr - ri * yi, xi = rr * yi + ri * yr;
        o_re[off] = xr;
        o_im[off] = xi;
        m = n - 1;
        for (; m - U + 1 >= 1; m -= U) {
            T y_r[U], y_i[U], q_r[U], q_i[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                long o2 = (long)(m - u) * W;
                y_r[u] = o_re[o2];
                y_i[u] = o_im[o2];
                q_r[u] = r_re[o2];
                q_i[u] = r_im[o2];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                T tr = y_r[u] - a * xr, ti = y_i[u] - a * xi;
                xr = q_r[u] * tr - q_i[u] * ti;
                xi = q_r[u] * ti + q_i[u] * tr;
                long o2 = (long)(m - u) * W;
                o_re[o2] = xr;
                o_im[o2] = xi;
            }
        }
        for (; m >= 0; --m) {
            long o2 = (long)m * W;
            T sr = (m == 0) ? s0r : a, si = (m == 0) ? s0i : T(0);
            T tr = o_re[o2] - (sr * xr - si * xi), ti = o_im[o2] - (sr * xi + si * xr);
            T q_r = r_re[o2], q_i = r_im[o2];
            xr = q_r * tr - q_i * ti;
            xi = q_r * ti + q_i * tr;
            o_re[o2] = xr;
            o_im[o2] = xi;
        }
    }
}

// ------------------------------------------------------------------ unfold helpers
// u(m, q) of right-hand side b, plane pl, from folded synthesis rows:
//   u_q = A_q + B_q, u_{n-q} = A_q - B_q (q < p), u_p = A_p, zero at q = 0, n.
template <class T>
__device__ inline double unfold_at(const T* __restrict__ u, const Fold& f, int b, int pl, int m, int q) {
    const int n = f.n, p = f.p;
    if (q <= 0 || q >= n) return 0.0;
    const T* row = u + (((long)b * 2 + pl) * (n + 1) + m) * f.W;
    if (q == p) return (double)row[p - 1];
    if (q < p) return (double)row[q - 1] + (double)row[f.P1 + q - 1];
    const int qq = n - q;
    return (double)row[qq - 1] - (double)row[f.P1 + qq - 1];
}

template <class T>
__device__ inline C64 unfold_c(const T* __restrict__ u, const Fold& f, int b, int m, int q) {
    return {unfold_at(u, f, b, 0, m, q), unfold_at(u, f, b, 1, m, q)};
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
__global__ void gather_q_kernel(const T* __restrict__ u, const float* __restrict__ du, Fold f,
                                const int* __restrict__ gm, const int* __restrict__ gq, int ng,
                                double* __restrict__ Q, int ldq, int col0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= ng) return;
    const int m = gm[i], q = gq[i];
    C64 v = unfold_c(u, f, b, m, q);
    if (du) v = cadd(v, unfold_c(du, f, b, m, q));
    double* o = Q + 2 * ((long)(col0 + b) * ldq + i);
    o[0] = -v.re;
    o[1] = -v.im;
}

// ------------------------------------------------------------------ unfold to grids
// out_b(m, q) = w_b(m, q) + alpha * u_b(m, q)  (w optional; complex interleaved FP64)
template <class T>
__global__ void unfold_grid_kernel(const T* __restrict__ u, const float* __restrict__ du, Fold f, double alpha,
                                   const double* w, long w_stride, double* out, long out_stride) {
    const int n = f.n;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y, b = blockIdx.z;
    if (q > n) return;
    const long node = (long)m * (n + 1) + q;
    C64 v = unfold_c(u, f, b, m, q);
    if (du) v = cadd(v, unfold_c(du, f, b, m, q));
    double re = alpha * v.re, im = alpha * v.im;
    if (w) {
        const double* wp = w + 2 * ((long)b * w_stride + node);
        re += wp[0];
        im += wp[1];
    }
    double* o = out + 2 * ((long)b * out_stride + node);
    o[0] = re;
    o[1] = im;
}

// ------------------------------------------------------------------ density on gamma for reconstruction
// w_b(gamma_i) = sum_col E(i, col) c_b(col)  (E real, c complex); w is pre-zeroed elsewhere.
__global__ void extend_density_kernel(const double* __restrict__ E, int ng, int ncol, const double* __restrict__ c,
                                      const int* __restrict__ gm, const int* __restrict__ gq, int n, double* w,
                                      long w_stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= ng) return;
    double re = 0.0, im = 0.0;
    const double* cb = c + 2 * (long)b * ncol;
    for (int col = 0; col < ncol; ++col) {
        double e = E[(long)col * ng + i];
        re += e * cb[2 * col];
        im += e * cb[2 * col + 1];
    }
    double* o = w + 2 * ((long)b * w_stride + (long)gm[i] * (n + 1) + gq[i]);
    o[0] = re;
    o[1] = im;
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

template <class T>
void launch_fold_rhs(const SrcDesc& s, int n, const Fold& f, StencilCoef sc, int R, bool cplx, T* out,
                     hipStream_t st) {
    check_batch(R);
    SrcEval ev{s, n, sc};
    const int bx = f.W < 256 ? f.W : 256;
    dim3 grid((f.W + bx - 1) / bx, n + 1, R);
    hipLaunchKernelGGL(fold_rhs_kernel<T>, grid, dim3(bx), 0, st, ev, f, cplx ? 2 : 1, out);
    MDP_HIP(hipGetLastError());
}

template <class T>
void launch_tridiag(const T* in, int planes_in, T* out, const T* fac, const T* colc, int n, const Fold& f, int R,
                    hipStream_t st) {
    check_batch(R);
    dim3 grid((f.W + 255) / 256, R);
    hipLaunchKernelGGL(tridiag_kernel<T>, grid, dim3(256), 0, st, in, planes_in, out, fac, colc, n, f.W, R);
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
void launch_gather_q(const T* u, const float* du, int n, const Fold& f, const int* gm, const int* gq, int ng, int R,
                     double* Q, int ldq, int col0, hipStream_t st) {
    (void)n;
    check_batch(R);
    dim3 grid((ng + 255) / 256, R);
    hipLaunchKernelGGL(gather_q_kernel<T>, grid, dim3(256), 0, st, u, du, f, gm, gq, ng, Q, ldq, col0);
    MDP_HIP(hipGetLastError());
}

template <class T>
void launch_unfold_grid(const T* u, const float* du, int n, const Fold& f, int R, const double* w, long w_stride,
                        double* out, long out_stride, hipStream_t st) {
    check_batch(R);
    double alpha = w ? -1.0 : 1.0;
    dim3 grid((n + 1 + 255) / 256, n + 1, R);
    hipLaunchKernelGGL(unfold_grid_kernel<T>, grid, dim3(256), 0, st, u, du, f, alpha, w, w_stride, out, out_stride);
    MDP_HIP(hipGetLastError());
}

void launch_extend_density(const double* E, int ng, int ncol, const double* c, int R, const int* gm,
                           const int* gq, int n, double* w, long w_stride, hipStream_t st) {
    check_batch(R);
    dim3 grid((ng + 255) / 256, R);
    hipLaunchKernelGGL(extend_density_kernel, grid, dim3(256), 0, st, E, ng, ncol, c, gm, gq, n, w, w_stride);
    MDP_HIP(hipGetLastError());
}

template void launch_fold_rhs<double>(const SrcDesc&, int, const Fold&, StencilCoef, int, bool, double*, hipStream_t);
template void launch_fold_rhs<float>(const SrcDesc&, int, const Fold&, StencilCoef, int, bool, float*, hipStream_t);
template void launch_tridiag<double>(const double*, int, double*, const double*, const double*, int, const Fold&, int,
                                     hipStream_t);
template void launch_tridiag<float>(const float*, int, float*, const float*, const float*, int, const Fold&, int,
                                    hipStream_t);
template void launch_gather_q<double>(const double*, const float*, int, const Fold&, const int*, const int*, int, int,
                                      double*, int, int, hipStream_t);
template void launch_gather_q<float>(const float*, const float*, int, const Fold&, const int*, const int*, int, int,
                                     double*, int, int, hipStream_t);
template void launch_unfold_grid<double>(const double*, const float*, int, const Fold&, int, const double*, long,
                                         double*, long, hipStream_t);
template void launch_unfold_grid<float>(const float*, const float*, int, const Fold&, int, const double*, long,
                                        double*, long, hipStream_t);

}  // namespace mdp
