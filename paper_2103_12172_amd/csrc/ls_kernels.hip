// Kernels of the interface least-squares solve (complex FP64).
//
// The reduced system Qbar c = Fbar (paper Sec. 3.3.3-3.5) is tall and skinny
// (sum |gamma_i| rows, 4 N M* columns).  It is factored as Qbar = Q R by
// Cholesky-QR passes whose work is almost entirely complex GEMM on the FP64
// matrix cores: Gram matrices, triangular inverses and the products with them.
// Kernels here: a general complex GEMM (op N / conjugate-transpose, split-K),
// the Cholesky + inverse of one diagonal block, and small assembly kernels.
#include "mdp_internal.h"

namespace mdp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma64(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// C(M x N) (+)= op(A)(M x K) op(B)(K x N), column-major, op in {N, C}.
// Workgroup tile 64 x 64, 4 waves of 32 x 32, K step 16; the K range of this
// workgroup is [kz*kchunk, min(K, (kz+1)*kchunk)).  With split-K (nsplit > 1)
// raw products go to P[kz] and a second kernel reduces them.
constexpr int ZBM = 64, ZBN = 64, ZBK = 16;

__global__ void __launch_bounds__(256)
zgemm_kernel(int opA, int opB, int M, int N, int K, const double2* __restrict__ A, int lda,
             const double2* __restrict__ B, int ldb, double2* __restrict__ C, int ldc, double2 alpha, double2 beta,
             int kchunk, double2* __restrict__ P, long pstride, int mtiles) {
    __shared__ double Ar[2][ZBK][ZBM + 2], Ai[2][ZBK][ZBM + 2];
    __shared__ double Br[2][ZBK][ZBN + 2], Bi[2][ZBK][ZBN + 2];
    const int tid = threadIdx.x;
    const int mt = blockIdx.x % mtiles, nt = blockIdx.x / mtiles;
    const int kz = blockIdx.y;
    const int m0 = mt * ZBM, n0 = nt * ZBN;
    const int kb = kz * kchunk, ke = min(K, kb + kchunk);
    const int wave = tid >> 6, lane = tid & 63, wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;

    d4 cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { cr[i][j] = d4{0, 0, 0, 0}; ci[i][j] = d4{0, 0, 0, 0}; }

    double2 ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int idx = tid + v * 256;
            int i, kk;
            if (opA == 0) { i = idx % ZBM; kk = idx / ZBM; } else { kk = idx % ZBK; i = idx / ZBK; }
            int gi = m0 + i, gk = k0 + kk;
            double2 a = make_double2(0.0, 0.0);
            if (gi < M && gk < ke) {
                a = (opA == 0) ? A[gi + (long)gk * lda] : A[gk + (long)gi * lda];
                if (opA) a.y = -a.y;
            }
            ra[v] = a;
            int j;
            if (opB == 0) { kk = idx % ZBK; j = idx / ZBK; } else { j = idx % ZBN; kk = idx / ZBN; }
            int gj = n0 + j;
            gk = k0 + kk;
            double2 b = make_double2(0.0, 0.0);
            if (gj < N && gk < ke) {
                b = (opB == 0) ? B[gk + (long)gj * ldb] : B[gj + (long)gk * ldb];
                if (opB) b.y = -b.y;
            }
            rb[v] = b;
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int idx = tid + v * 256;
            int i, kk, j;
            if (opA == 0) { i = idx % ZBM; kk = idx / ZBM; } else { kk = idx % ZBK; i = idx / ZBK; }
            Ar[buf][kk][i] = ra[v].x;
            Ai[buf][kk][i] = ra[v].y;
            if (opB == 0) { kk = idx % ZBK; j = idx / ZBK; } else { j = idx % ZBN; kk = idx / ZBN; }
            Br[buf][kk][j] = rb[v].x;
            Bi[buf][kk][j] = rb[v].y;
        }
    };

    if (kb < ke) {
        gload(kb);
        lstore(0);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += ZBK) {
        const bool more = k0 + ZBK < ke;
        if (more) gload(k0 + ZBK);
#pragma unroll
        for (int kk = 0; kk < ZBK / 4; ++kk) {
            double ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ar[i] = Ar[buf][kk * 4 + lk][wm * 32 + i * 16 + lr];
                ai[i] = Ai[buf][kk * 4 + lk][wm * 32 + i * 16 + lr];
                br[i] = Br[buf][kk * 4 + lk][wn * 32 + i * 16 + lr];
                bi[i] = Bi[buf][kk * 4 + lk][wn * 32 + i * 16 + lr];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    cr[i][j] = mfma64(ar[i], br[j], cr[i][j]);
                    cr[i][j] = mfma64(-ai[i], bi[j], cr[i][j]);
                    ci[i][j] = mfma64(ar[i], bi[j], ci[i][j]);
                    ci[i][j] = mfma64(ai[i], br[j], ci[i][j]);
                }
        }
        if (more) lstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int gi = m0 + wm * 32 + i * 16 + lk + 4 * r;   // f64 MFMA D rows: (lane>>4) + 4r
                int gj = n0 + wn * 32 + j * 16 + lr;
                if (gi >= M || gj >= N) continue;
                double vr = cr[i][j][r], vi = ci[i][j][r];
                if (P) {
                    P[kz * pstride + gi + (long)gj * M] = make_double2(vr, vi);
                } else {
                    double2 o = make_double2(alpha.x * vr - alpha.y * vi, alpha.x * vi + alpha.y * vr);
                    double2* cp = C + gi + (long)gj * ldc;
                    if (beta.x != 0.0 || beta.y != 0.0) {
                        double2 c = *cp;
                        o.x += beta.x * c.x - beta.y * c.y;
                        o.y += beta.x * c.y + beta.y * c.x;
                    }
                    *cp = o;
                }
            }
}

__global__ void zgemm_reduce_kernel(int M, int N, int nsplit, const double2* __restrict__ P, long pstride,
                                    double2* __restrict__ C, int ldc, double2 alpha, double2 beta) {
    long total = (long)M * N;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        int i = (int)(t % M), j = (int)(t / M);
        double sr = 0.0, si = 0.0;
        for (int s = 0; s < nsplit; ++s) {
            double2 v = P[s * pstride + t];
            sr += v.x;
            si += v.y;
        }
        double2 o = make_double2(alpha.x * sr - alpha.y * si, alpha.x * si + alpha.y * sr);
        double2* cp = C + i + (long)j * ldc;
        if (beta.x != 0.0 || beta.y != 0.0) {
            double2 c = *cp;
            o.x += beta.x * c.x - beta.y * c.y;
            o.y += beta.x * c.y + beta.y * c.x;
        }
        *cp = o;
    }
}

// Cholesky of one Hermitian diagonal block (lower: G = L L^H) and the inverse of
// its factor, in LDS.  G (nb x nb, leading dim ldg) is read; L goes to Lout
// (ld ldl, upper part zeroed) and L^{-1} to Linv (ld ldi).  A non-positive pivot
// sets *info to its 1-based index (first failure wins) and the block is then
// not usable.  `shift` is added to the diagonal before factoring.
template <int NB>
__global__ void __launch_bounds__(256)
chol_block_kernel(const double2* __restrict__ G, int ldg, int nb, double shift, double2* __restrict__ Lout, int ldl,
                  double2* __restrict__ Linv, int ldi, int* info, int base) {
    __shared__ double2 S[NB][NB + 1];
    __shared__ double2 X[NB][NB + 1];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    for (int t = tid; t < NB * NB; t += 256) {
        int i = t % NB, j = t / NB;
        double2 v = make_double2(0.0, 0.0);
        if (i < nb && j < nb) v = G[i + (long)j * ldg];
        else if (i == j) v = make_double2(1.0, 0.0);  // identity padding keeps the factor regular
        if (i == j && i < nb) v.x += shift;
        S[i][j] = v;
    }
    __syncthreads();
    for (int k = 0; k < NB; ++k) {
        // pivot
        if (tid == 0) {
            double d = S[k][k].x;
            if (!(d > 0.0)) {
                if (!bad) bad = k + 1;
                d = 1.0;
            }
            S[k][k] = make_double2(sqrt(d), 0.0);
        }
        __syncthreads();
        double dk = S[k][k].x;
        for (int i = k + 1 + tid; i < NB; i += 256) {
            S[i][k].x /= dk;
            S[i][k].y /= dk;
        }
        __syncthreads();
        // trailing update of the lower triangle: S(i,j) -= L(i,k) conj(L(j,k)), k < j <= i
        const int r = NB - k - 1;
        for (int t = tid; t < r * r; t += 256) {
            int i = k + 1 + t % r, j = k + 1 + t / r;
            if (j > i) continue;
            double2 a = S[i][k], b = S[j][k];
            S[i][j].x -= a.x * b.x + a.y * b.y;
            S[i][j].y -= a.y * b.x - a.x * b.y;
        }
        __syncthreads();
    }
    // inverse of the lower-triangular factor, one column per thread: L X = I
    if (tid < NB) {
        const int c = tid;
        for (int i = 0; i < NB; ++i) {
            if (i < c) { X[i][c] = make_double2(0.0, 0.0); continue; }
            double sr = (i == c) ? 1.0 : 0.0, si = 0.0;
            for (int k = c; k < i; ++k) {
                double2 l = S[i][k], x = X[k][c];
                sr -= l.x * x.x - l.y * x.y;
                si -= l.x * x.y + l.y * x.x;
            }
            double d = S[i][i].x;
            X[i][c] = make_double2(sr / d, si / d);
        }
    }
    __syncthreads();
    for (int t = tid; t < nb * nb; t += 256) {
        int i = t % nb, j = t / nb;
        Lout[i + (long)j * ldl] = (j <= i) ? S[i][j] : make_double2(0.0, 0.0);
        Linv[i + (long)j * ldi] = (j <= i) ? X[i][j] : make_double2(0.0, 0.0);
    }
    if (tid == 0 && bad && info) atomicCAS(info, 0, base + bad);
}

// Qbar(r, c) for rows of subdomain s: sum of up to two weighted columns of Q_s.
// colmap[s*ncol + c] = (colA, colB, -, -) with -1 = absent; coefs likewise (2 per entry).
__global__ void assemble_qbar_kernel(const double2* const* __restrict__ Qsrc, const int* __restrict__ qld, int n_sub,
                                     const int* __restrict__ row_off, const int4* __restrict__ colmap,
                                     const double2* __restrict__ coefs, int ncol, double2* __restrict__ Qbar,
                                     int ldq) {
    const int c = blockIdx.y;
    const int total_rows = row_off[n_sub];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < total_rows; r += gridDim.x * blockDim.x) {
        int s = 0;
        while (r >= row_off[s + 1]) ++s;
        const int rl = r - row_off[s];
        const int4 cm = colmap[(long)s * ncol + c];
        double2 v = make_double2(0.0, 0.0);
        if (cm.x >= 0) {
            double2 q = Qsrc[s][rl + (long)cm.x * qld[s]], w = coefs[2 * ((long)s * ncol + c)];
            v.x += w.x * q.x - w.y * q.y;
            v.y += w.x * q.y + w.y * q.x;
        }
        if (cm.y >= 0) {
            double2 q = Qsrc[s][rl + (long)cm.y * qld[s]], w = coefs[2 * ((long)s * ncol + c) + 1];
            v.x += w.x * q.x - w.y * q.y;
            v.y += w.x * q.y + w.y * q.x;
        }
        Qbar[r + (long)c * ldq] = v;
    }
}

// F(r) = -sum_k Q_s(rl, kcol[k]) * kval[k] over the known coefficients of subdomain s.
__global__ void known_rhs_kernel(const double2* const* __restrict__ Qsrc, const int* __restrict__ qld, int n_sub,
                                 const int* __restrict__ row_off, const int* __restrict__ kcol,
                                 const double2* __restrict__ kval, const int* __restrict__ koff,
                                 double2* __restrict__ F) {
    const int total_rows = row_off[n_sub];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < total_rows; r += gridDim.x * blockDim.x) {
        int s = 0;
        while (r >= row_off[s + 1]) ++s;
        const int rl = r - row_off[s];
        double sr = 0.0, si = 0.0;
        for (int k = koff[s]; k < koff[s + 1]; ++k) {
            double2 q = Qsrc[s][rl + (long)kcol[k] * qld[s]], w = kval[k];
            sr += w.x * q.x - w.y * q.y;
            si += w.x * q.y + w.y * q.x;
        }
        F[r] = make_double2(-sr, -si);
    }
}

__global__ void col_norms_kernel(const double2* __restrict__ A, int m, int lda, double* __restrict__ out) {
    const int c = blockIdx.x;
    __shared__ double red[256];
    double s = 0.0;
    for (int r = threadIdx.x; r < m; r += 256) {
        double2 v = A[r + (long)c * lda];
        s += v.x * v.x + v.y * v.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sqrt(red[0]);
}

__global__ void scale_cols_kernel(double2* A, int m, int n, int lda, const double* __restrict__ s, int invert) {
    long total = (long)m * n;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        int r = (int)(t % m), c = (int)(t / m);
        double f = invert ? (s[c] > 0.0 ? 1.0 / s[c] : 0.0) : s[c];
        double2* p = A + r + (long)c * lda;
        p->x *= f;
        p->y *= f;
    }
}

__global__ void fill_kernel(double* p, long n, double v) {
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) p[t] = v;
}

inline unsigned blocks_for(long total) {
    long g = (total + 255) / 256;
    if (g > (1 << 16)) g = 1 << 16;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

void launch_zgemm(char opA, char opB, int m, int n, int k, double2 alpha, const double2* A, int lda,
                  const double2* B, int ldb, double2 beta, double2* C, int ldc, DevBuf& P, hipStream_t st) {
    if (m <= 0 || n <= 0) return;
    const int oa = (opA == 'C') ? 1 : 0, ob = (opB == 'C') ? 1 : 0;
    const int mt = (m + ZBM - 1) / ZBM, nt = (n + ZBN - 1) / ZBN;
    const int tiles = mt * nt;
    int nsplit = 1;
    if (k > 0 && tiles < 512) {
        nsplit = (512 + tiles - 1) / tiles;
        nsplit = std::min(nsplit, std::max(1, k / 128));
        nsplit = std::min(nsplit, 64);
    }
    int kchunk = (k + nsplit - 1) / nsplit;
    kchunk = (kchunk + ZBK - 1) / ZBK * ZBK;
    if (kchunk < ZBK) kchunk = ZBK;
    nsplit = (k > 0) ? (k + kchunk - 1) / kchunk : 1;
    if (nsplit <= 1) {
        hipLaunchKernelGGL(zgemm_kernel, dim3(tiles, 1), dim3(256), 0, st, oa, ob, m, n, k, A, lda, B, ldb, C, ldc,
                           alpha, beta, kchunk, (double2*)nullptr, 0L, mt);
        MDP_HIP(hipGetLastError());
        return;
    }
    const long pstride = (long)m * n;
    const size_t need = (size_t)pstride * nsplit * sizeof(double2);
    if (need > P.bytes) {   // never free a buffer earlier kernels may still read
        MDP_HIP(hipDeviceSynchronize());
        P.reserve(need);
    }
    hipLaunchKernelGGL(zgemm_kernel, dim3(tiles, nsplit), dim3(256), 0, st, oa, ob, m, n, k, A, lda, B, ldb, C, ldc,
                       alpha, beta, kchunk, P.as<double2>(), pstride, mt);
    MDP_HIP(hipGetLastError());
    hipLaunchKernelGGL(zgemm_reduce_kernel, dim3(blocks_for(pstride)), dim3(256), 0, st, m, n, nsplit,
                       P.as<double2>(), pstride, C, ldc, alpha, beta);
    MDP_HIP(hipGetLastError());
}

void launch_chol_block(const double2* G, int ldg, int nb, double shift, double2* L, int ldl, double2* Linv, int ldi,
                       int* info, int base, hipStream_t st) {
    if (nb <= 32)
        hipLaunchKernelGGL(chol_block_kernel<32>, dim3(1), dim3(256), 0, st, G, ldg, nb, shift, L, ldl, Linv, ldi,
                           info, base);
    else if (nb <= 64)
        hipLaunchKernelGGL(chol_block_kernel<64>, dim3(1), dim3(256), 0, st, G, ldg, nb, shift, L, ldl, Linv, ldi,
                           info, base);
    else
        throw Error(MDP_ERR_ARG, "Cholesky block too large");
    MDP_HIP(hipGetLastError());
}

void launch_assemble_qbar(const double2* const* Qsrc, const int* qld, int n_sub, const int* row_off, int total_rows,
                          const int4* colmap, const double2* coefs, int ncol, double2* Qbar, int ldq, hipStream_t st) {
    dim3 grid(std::max(1, std::min((total_rows + 255) / 256, 1024)), ncol);
    hipLaunchKernelGGL(assemble_qbar_kernel, grid, dim3(256), 0, st, Qsrc, qld, n_sub, row_off, colmap, coefs, ncol,
                       Qbar, ldq);
    MDP_HIP(hipGetLastError());
}

void launch_known_rhs(const double2* const* Qsrc, const int* qld, int n_sub, const int* row_off, int total_rows,
                      const int* kcol, const double2* kval, const int* koff, double2* F, hipStream_t st) {
    hipLaunchKernelGGL(known_rhs_kernel, dim3(blocks_for(total_rows)), dim3(256), 0, st, Qsrc, qld, n_sub, row_off,
                       kcol, kval, koff, F);
    MDP_HIP(hipGetLastError());
}

void launch_col_norms(const double2* A, int m, int n, int lda, double* out, hipStream_t st) {
    hipLaunchKernelGGL(col_norms_kernel, dim3(n), dim3(256), 0, st, A, m, lda, out);
    MDP_HIP(hipGetLastError());
}

void launch_scale_cols(double2* A, int m, int n, int lda, const double* s, int invert, hipStream_t st) {
    hipLaunchKernelGGL(scale_cols_kernel, dim3(blocks_for((long)m * n)), dim3(256), 0, st, A, m, n, lda, s, invert);
    MDP_HIP(hipGetLastError());
}

void launch_fill(double* p, long n, double v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n)), dim3(256), 0, st, p, n, v);
    MDP_HIP(hipGetLastError());
}

}  // namespace mdp
