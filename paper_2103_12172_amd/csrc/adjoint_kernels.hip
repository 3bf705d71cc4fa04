// Kernels of the receiver-functional gradient (reverse mode through the three
// steps of paper Sec. 3.5, f = 0): the adjoint of the reconstruction read on
// gamma, the adjoint of the coefficient expansion, the boundary-data gradient,
// and the k^2 directional derivative of an AP solve's right-hand side.
// Grids are complex interleaved FP64, (n+1)^2 per function, index m*(n+1)+q.
#include "mdp_internal.h"

namespace mdp {
namespace {

__device__ inline double2 wave_sum(double2 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    return v;
}

// sum over the 256 threads of a workgroup (result valid in thread 0)
__device__ inline double2 block_sum(double2 v) {
    __shared__ double2 part[4];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    if (threadIdx.x == 0)
        for (int i = 0; i < 4; ++i) {
            s.x += part[i].x;
            s.y += part[i].y;
        }
    return s;
}

__device__ inline bool in_box(int m, int q, int m_lo, int m_hi, int q_lo, int q_hi) {
    return m >= m_lo && m <= m_hi && q >= q_lo && q <= q_hi;
}

__global__ void scatter_values_kernel(const long* __restrict__ off, const double* __restrict__ val, int count,
                                      double* grids) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    grids[2 * off[t]] = val[2 * t];
    grids[2 * off[t] + 1] = val[2 * t + 1];
}

// wbar_b(i) = ubar_b(node_i) - sum_r c(r - node_i) lambda_b(r) over the 3x3 neighbours r in M+
__global__ void gamma_adjoint_kernel(const double* __restrict__ ubar, const double* __restrict__ lambda,
                                     const long* __restrict__ goff, int n, StencilCoef sc, int m_lo, int m_hi,
                                     int q_lo, int q_hi, const int* __restrict__ gm, const int* __restrict__ gq,
                                     int ng, double* __restrict__ wbar, long wbar_stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= ng) return;
    const int m = gm[i], q = gq[i];
    const double* U = ubar + 2 * goff[b];
    const double* Lm = lambda + 2 * goff[b];
    double re = U[2 * ((long)m * (n + 1) + q)], im = U[2 * ((long)m * (n + 1) + q) + 1];
    for (int dm = -1; dm <= 1; ++dm)
        for (int dq = -1; dq <= 1; ++dq) {
            const int mm = m + dm, qq = q + dq;
            if (!in_box(mm, qq, m_lo, m_hi, q_lo, q_hi)) continue;
            const double c = (dm == 0 && dq == 0) ? sc.c0 : ((dm == 0 || dq == 0) ? sc.ce : sc.cc);
            const long node = (long)mm * (n + 1) + qq;
            re -= c * Lm[2 * node];
            im -= c * Lm[2 * node + 1];
        }
    wbar[2 * ((long)b * wbar_stride + i)] = re;
    wbar[2 * ((long)b * wbar_stride + i) + 1] = im;
}

// cbar_b(col) = sum_i E(i, col) wbar_b(i): one workgroup per (col, b)
__global__ void __launch_bounds__(256)
et_apply_kernel(const double* __restrict__ E, int ng, int ncol, const double* __restrict__ wbar, long wbar_stride,
                const int* __restrict__ cidx, double* __restrict__ cbar) {
    const int col = blockIdx.x, b = blockIdx.y;
    const double* e = E + (long)col * ng;
    const double* wb = wbar + 2 * (long)b * wbar_stride;
    double2 s = make_double2(0.0, 0.0);
    for (int i = threadIdx.x; i < ng; i += 256) {
        const double v = e[i];
        s.x += v * wb[2 * i];
        s.y += v * wb[2 * i + 1];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) {
        double* o = cbar + 2 * ((long)cidx[b] * ncol + col);
        o[0] = s.x;
        o[1] = s.y;
    }
}

// xbar[src[e]] += conj(coef[e]) cbar[e]; an unknown receives at most two terms, whose
// sum does not depend on their order
__global__ void expand_adj_kernel(int n, const int* __restrict__ src, const double2* __restrict__ coef,
                                  const double2* __restrict__ cbar, double2* xbar) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int s = src[e];
    if (s < 0) return;
    const double2 a = coef[e], c = cbar[e];
    double* o = reinterpret_cast<double*>(xbar + s);
    atomicAdd(&o[0], a.x * c.x + a.y * c.y);
    atomicAdd(&o[1], a.x * c.y - a.y * c.x);
}

// one workgroup per known coefficient t
__global__ void __launch_bounds__(256)
data_grad_kernel(const double2* const* __restrict__ Q, const int* __restrict__ rows, const int* __restrict__ kcol,
                 const long* __restrict__ roff, const int* __restrict__ eidx, const double* __restrict__ div,
                 const double2* __restrict__ cbar, const double2* __restrict__ Fb, double2* __restrict__ out) {
    const int t = blockIdx.x;
    const int nr = rows[t];
    const double2* q = Q[t] + (long)kcol[t] * nr;
    const double2* f = Fb + roff[t];
    double2 s = make_double2(0.0, 0.0);
    for (int r = threadIdx.x; r < nr; r += 256) {   // conj(Q) Fb
        const double2 a = q[r], b = f[r];
        s.x += a.x * b.x + a.y * b.y;
        s.y += a.x * b.y - a.y * b.x;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) {
        const double2 c = cbar[eidx[t]];
        const double dv = div[t];
        out[t] = make_double2((c.x - s.x) / dv, (c.y - s.y) / dv);
    }
}

// h_b = -dA v_b + (dL w_b + L dw_b)|M+ at node (m, q), m = 0..n, q = 0..n (zero at q = 0, n)
__global__ void jvp_rhs_kernel(const double* __restrict__ v, const double* __restrict__ w,
                               const double* __restrict__ dw, const long* __restrict__ goff, int n, double h,
                               double k, StencilCoef sc, StencilCoef dsc, int m_lo, int m_hi, int q_lo, int q_hi,
                               double* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y, b = blockIdx.z;
    if (q > n) return;
    const long base = 2 * goff[b];
    const double* V = v + base;
    auto at = [&](const double* g, int mm, int qq) -> double2 {
        if (qq <= 0 || qq >= n) return make_double2(0.0, 0.0);
        const long node = (long)mm * (n + 1) + qq;
        return make_double2(g[2 * node], g[2 * node + 1]);
    };
    double re = 0.0, im = 0.0;
    if (q > 0 && q < n) {
        if (m == 0 || m == n) {
            // derivative of the Sommerfeld-type row: (h/24) D +- i [dmid A_q + dside (A_{q-1} + A_{q+1})]
            const int mo = (m == 0) ? 0 : n, mi = (m == 0) ? 1 : n - 1;
            const double sgn = (m == 0) ? -1.0 : 1.0;
            const double wA = 1.0 + k * k * h * h / 8.0, wA2 = 1.0 / 8.0;
            const double dmid = (wA - 2.0 * wA2) / (2.0 * k) + k * h * h / 8.0, dside = wA2 / (2.0 * k);
            const double2 uo = at(V, mo, q), ui = at(V, mi, q);
            const double Dr = (m == 0) ? (ui.x - uo.x) : (uo.x - ui.x);
            const double Di = (m == 0) ? (ui.y - uo.y) : (uo.y - ui.y);
            double Ar = 0.0, Ai = 0.0;
            for (int dq = -1; dq <= 1; ++dq) {
                const double2 a = at(V, mo, q + dq), c = at(V, mi, q + dq);
                const double wgt = (dq == 0 ? dmid : dside) * 0.5;
                Ar += wgt * (a.x + c.x);
                Ai += wgt * (a.y + c.y);
            }
            // value = (h/24) D + sgn i A
            re = -(h / 24.0 * Dr - sgn * Ai);
            im = -(h / 24.0 * Di + sgn * Ar);
        } else {
            const double2 c = at(V, m, q);
            const double2 e0 = at(V, m + 1, q), e1 = at(V, m - 1, q), e2 = at(V, m, q + 1), e3 = at(V, m, q - 1);
            const double2 k0 = at(V, m + 1, q + 1), k1 = at(V, m - 1, q + 1), k2 = at(V, m + 1, q - 1),
                          k3 = at(V, m - 1, q - 1);
            re = -(dsc.c0 * c.x + dsc.ce * (e0.x + e1.x + e2.x + e3.x) + dsc.cc * (k0.x + k1.x + k2.x + k3.x));
            im = -(dsc.c0 * c.y + dsc.ce * (e0.y + e1.y + e2.y + e3.y) + dsc.cc * (k0.y + k1.y + k2.y + k3.y));
            if (in_box(m, q, m_lo, m_hi, q_lo, q_hi)) {
                const double* Wg = w + base;
                const double* Dg = dw + base;
                auto st9 = [&](const double* g, const StencilCoef& s, double& ar, double& ai) {
                    const double2 cc = at(g, m, q);
                    const double2 a0 = at(g, m + 1, q), a1 = at(g, m - 1, q), a2 = at(g, m, q + 1),
                                  a3 = at(g, m, q - 1);
                    const double2 b0 = at(g, m + 1, q + 1), b1 = at(g, m - 1, q + 1), b2 = at(g, m + 1, q - 1),
                                  b3 = at(g, m - 1, q - 1);
                    ar += s.c0 * cc.x + s.ce * (a0.x + a1.x + a2.x + a3.x) + s.cc * (b0.x + b1.x + b2.x + b3.x);
                    ai += s.c0 * cc.y + s.ce * (a0.y + a1.y + a2.y + a3.y) + s.cc * (b0.y + b1.y + b2.y + b3.y);
                };
                st9(Wg, dsc, re, im);
                st9(Dg, sc, re, im);
            }
        }
    }
    const long node = (long)m * (n + 1) + q;
    out[base + 2 * node] = re;
    out[base + 2 * node + 1] = im;
}

__global__ void __launch_bounds__(256)
kappa_dot_kernel(const double* __restrict__ yf, const double* __restrict__ yz, const double* __restrict__ dwf,
                 const int* __restrict__ gm, const int* __restrict__ gq, int ng, int n, const double2* __restrict__ Fb,
                 const double2* __restrict__ r, long r0, const long* __restrict__ rcv_node,
                 const double* __restrict__ rcv_val, int rcv_count, double2* __restrict__ out) {
    double2 s = make_double2(0.0, 0.0);
    for (int g = threadIdx.x; g < ng; g += 256) {
        const long node = (long)gm[g] * (n + 1) + gq[g];
        const double2 f = Fb[r0 + g], rr = r[r0 + g];
        const double ar = yf[2 * node], ai = yf[2 * node + 1], br = yz[2 * node], bi = yz[2 * node + 1];
        // conj(f) yf - conj(r) yz
        s.x += f.x * ar + f.y * ai - (rr.x * br + rr.y * bi);
        s.y += f.x * ai - f.y * ar - (rr.x * bi - rr.y * br);
    }
    for (int t = threadIdx.x; t < rcv_count; t += 256) {
        const long node = rcv_node[t];
        const double ur = rcv_val[2 * t], ui = rcv_val[2 * t + 1];
        const double dr = dwf[2 * node] - yf[2 * node], di = dwf[2 * node + 1] - yf[2 * node + 1];
        s.x += ur * dr + ui * di;
        s.y += ur * di - ui * dr;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace

void launch_scatter_values(const long* off, const double* val, int count, double* grids, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(scatter_values_kernel, dim3((count + 255) / 256), dim3(256), 0, st, off, val, count, grids);
    MDP_HIP(hipGetLastError());
}

void launch_gamma_adjoint(const double* ubar, const double* lambda, const long* goff, int R, int n, StencilCoef sc,
                          int m_lo, int m_hi, int q_lo, int q_hi, const int* gm, const int* gq, int ng, double* wbar,
                          long wbar_stride, hipStream_t st) {
    if (R <= 0 || ng <= 0) return;
    hipLaunchKernelGGL(gamma_adjoint_kernel, dim3((ng + 255) / 256, R), dim3(256), 0, st, ubar, lambda, goff, n, sc,
                       m_lo, m_hi, q_lo, q_hi, gm, gq, ng, wbar, wbar_stride);
    MDP_HIP(hipGetLastError());
}

void launch_et_apply(const double* E, int ng, int ncol, const double* wbar, long wbar_stride, int R, const int* cidx,
                     double* cbar, hipStream_t st) {
    if (R <= 0 || ncol <= 0) return;
    hipLaunchKernelGGL(et_apply_kernel, dim3(ncol, R), dim3(256), 0, st, E, ng, ncol, wbar, wbar_stride, cidx, cbar);
    MDP_HIP(hipGetLastError());
}

void launch_expand_adj(int n, const int* src, const double2* coef, const double2* cbar, double2* xbar, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(expand_adj_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, src, coef, cbar, xbar);
    MDP_HIP(hipGetLastError());
}

void launch_data_grad(int count, const double2* const* Q, const int* rows, const int* kcol, const long* roff,
                      const int* eidx, const double* div, const double2* cbar, const double2* Fb, double2* out,
                      hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(data_grad_kernel, dim3(count), dim3(256), 0, st, Q, rows, kcol, roff, eidx, div, cbar, Fb, out);
    MDP_HIP(hipGetLastError());
}

void launch_jvp_rhs(const double* v, const double* w, const double* dw, const long* goff, int R, int n, double h,
                    double k, StencilCoef sc, StencilCoef dsc, int m_lo, int m_hi, int q_lo, int q_hi, double* out,
                    hipStream_t st) {
    if (R <= 0) return;
    hipLaunchKernelGGL(jvp_rhs_kernel, dim3((n + 1 + 255) / 256, n + 1, R), dim3(256), 0, st, v, w, dw, goff, n, h, k,
                       sc, dsc, m_lo, m_hi, q_lo, q_hi, out);
    MDP_HIP(hipGetLastError());
}

void launch_kappa_dot(const double* yf, const double* yz, const double* dwf, const int* gm, const int* gq, int ng,
                      int n, const double2* Fb, const double2* r, long r0, const long* rcv_node, const double* rcv_val,
                      int rcv_count, double2* out, hipStream_t st) {
    hipLaunchKernelGGL(kappa_dot_kernel, dim3(1), dim3(256), 0, st, yf, yz, dwf, gm, gq, ng, n, Fb, r, r0, rcv_node,
                       rcv_val, rcv_count, out);
    MDP_HIP(hipGetLastError());
}

}  // namespace mdp
