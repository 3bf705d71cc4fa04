// Kernels of the interface least-squares solve (complex FP64).
//
// The reduced system Qbar c = Fbar (Sec. 3.3.3-3.5) is tall and skinny (sum |gamma_i|
// rows, 4 N M* columns).  It is solved by the corrected semi-normal equations: the
// Gram matrix G = Qbar^* Qbar of the column-equilibrated packed blocks (split-K
// complex GEMM on the FP64 matrix cores), its Cholesky factor L together with
// L^{-1} (dense for one matrix, multifrontal over the subdomains' elimination tree
// for many: batched panel and update launches per 64 columns), and normal solves
// G dx = Qbar^* r with the explicit inverses, refined on the residual of the
// packed blocks.  Kernels here: the complex GEMM and Gram batch (three real MFMA
// products per complex product), the blocked Cholesky-with-inverse steps, the
// multifrontal assembly and substitutions, and the packed-block products (A x,
// A^* y, a refinement step's residual and A^* r in one pass, column norms, assembly).
#include "mdp_internal.h"

namespace mdp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma64(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// The dispatcher deals consecutive workgroups round-robin to the eight XCDs.  For a batch
// launch (x, y = tile of a batch entry, z = entry) renumber the workgroups so that XCD x
// runs the x-th eighth of the launch in order (a remainder keeps its place): every tile of
// one entry then runs on the same XCD, and the tiles sharing an operand block read it
// through one L2 (dealt as launched, every XCD would stream every entry's operands).
__device__ inline long xcd_grouped(long lin, long total) {
    const long per = total >> 3;
    return lin < per * 8 ? (lin & 7) * per + (lin >> 3) : lin;
}

// C(M x N) (+)= op(A)(M x K) op(B)(K x N), column-major, op in {N, C}.
// Workgroup tile ZBM x ZBM (32 or 64), 4 waves of ZBM/2 x ZBM/2, K step 16; the K
// range of this workgroup is [kz*kchunk, min(K, (kz+1)*kchunk)).  With split-K
// (nsplit > 1) raw products go to P[kz] and a second kernel reduces them.
// Each complex product takes three real MFMA products instead of four (the 3M form:
// ar br, ai bi and (ar + ai)(br + bi); re = P1 - P2, im = P3 - P1 - P2), normwise as
// accurate as the four-product form up to a small constant factor.
constexpr int ZBK = 16;

// tri: 0 = full; 1 = only tiles touching the lower triangle of C are computed
// (C Hermitian, lower part used); 2 = op(B) is upper triangular, so column tile
// n0 only needs k < n0 + 64.
// With zb set, blockIdx.z selects a batch entry whose A (= B), sizes, K chunk and
// split-K partial area replace the scalar arguments (Gram products A^* A).
template <int ZBM>
__global__ void __launch_bounds__(256)
zgemm_kernel(int opA, int opB, int M, int N, int K, const double2* __restrict__ A, int lda,
             const double2* __restrict__ B, int ldb, double2* __restrict__ C, int ldc, double2 alpha, double2 beta,
             int kchunk, double2* __restrict__ P, long pstride, int mtiles, int tri, const ZBatch* __restrict__ zb) {
    constexpr int ZBN = ZBM;
    int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    if (zb) {   // every tile of one Gram product on one XCD
        const long w = xcd_grouped(bx + (long)gridDim.x * (by + (long)gridDim.y * bz),
                                   (long)gridDim.x * gridDim.y * gridDim.z);
        bx = (int)(w % gridDim.x);
        const long r = w / gridDim.x;
        by = (int)(r % gridDim.y);
        bz = (int)(r / gridDim.y);
        const ZBatch e = zb[bz];
        A = B = e.A;
        M = N = e.n;
        K = e.k;
        lda = ldb = e.k;
        kchunk = e.kchunk;
        P += e.poff;
        pstride = (long)e.n * e.n;
        mtiles = (e.n + ZBM - 1) / ZBM;
        if (bx >= mtiles * mtiles) return;
    }
    constexpr int WT = ZBM / 2;          // wave tile (2 x 2 waves)
    constexpr int TT = WT / 16;          // 16x16 MFMA blocks per wave side
    constexpr int NL = ZBM * ZBK / 256;  // complex elements per thread per tile
    // operands as interleaved complex (one 16-byte read per operand and lane: a quarter-wave
    // reads 16 consecutive entries, all 64 banks once; the row padding keeps the k-major
    // stores conflict-free too)
    __shared__ double2 As[2][ZBK][ZBM + 1];
    __shared__ double2 Bs[2][ZBK][ZBN + 1];
    const int tid = threadIdx.x;
    const int mt = bx % mtiles, nt = bx / mtiles;
    const int kz = by;
    const int m0 = mt * ZBM, n0 = nt * ZBN;
    if (tri == 1 && m0 + ZBM <= n0) return;
    const int kb = kz * kchunk;
    int ke = min(K, kb + kchunk);
    if (tri == 2) ke = min(ke, n0 + ZBN);
    const int wave = tid >> 6, lane = tid & 63, wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;

    d4 c1[TT][TT], c2[TT][TT], c3[TT][TT];
#pragma unroll
    for (int i = 0; i < TT; ++i)
#pragma unroll
        for (int j = 0; j < TT; ++j) { c1[i][j] = d4{0, 0, 0, 0}; c2[i][j] = d4{0, 0, 0, 0}; c3[i][j] = d4{0, 0, 0, 0}; }

    double2 ra[NL], rb[NL];
    auto gload = [&](int k0) {
#pragma unroll
        for (int v = 0; v < NL; ++v) {
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
        for (int v = 0; v < NL; ++v) {
            int idx = tid + v * 256;
            int i, kk, j;
            if (opA == 0) { i = idx % ZBM; kk = idx / ZBM; } else { kk = idx % ZBK; i = idx / ZBK; }
            As[buf][kk][i] = ra[v];
            if (opB == 0) { kk = idx % ZBK; j = idx / ZBK; } else { j = idx % ZBN; kk = idx / ZBN; }
            Bs[buf][kk][j] = rb[v];
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
            double ar[TT], ai[TT], br[TT], bi[TT];
#pragma unroll
            for (int i = 0; i < TT; ++i) {
                const double2 a = As[buf][kk * 4 + lk][wm * WT + i * 16 + lr];
                const double2 b = Bs[buf][kk * 4 + lk][wn * WT + i * 16 + lr];
                ar[i] = a.x;
                ai[i] = a.y;
                br[i] = b.x;
                bi[i] = b.y;
            }
#pragma unroll
            for (int i = 0; i < TT; ++i)
#pragma unroll
                for (int j = 0; j < TT; ++j) {
                    c1[i][j] = mfma64(ar[i], br[j], c1[i][j]);
                    c2[i][j] = mfma64(ai[i], bi[j], c2[i][j]);
                    c3[i][j] = mfma64(ar[i] + ai[i], br[j] + bi[j], c3[i][j]);
                }
        }
        if (more) lstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < TT; ++i)
#pragma unroll
        for (int j = 0; j < TT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int gi = m0 + wm * WT + i * 16 + lk + 4 * r;   // f64 MFMA D rows: (lane>>4) + 4r
                int gj = n0 + wn * WT + j * 16 + lr;
                if (gi >= M || gj >= N) continue;
                double vr = c1[i][j][r] - c2[i][j][r], vi = c3[i][j][r] - c1[i][j][r] - c2[i][j][r];
                if (P) {
                    P[kz * pstride + gi + (long)gj * M] = make_double2(vr, vi);   // zero if this K range was empty
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

// The Gram batch A_b^* A_b (A_b column-major k x n, ld k): rectangular GM x GN workgroup tiles
// (rows i of A^*, columns j), only those touching the lower triangle; 4 waves of
// GM/2 x GN/2 (two 16x16 MFMA blocks sharing the B fragment when GM = 64), K step 16 through
// double-buffered LDS with the global loads of the two following K steps in flight (one step
// in flight left the batch latency-bound: 5.1 against 3.9 ms on the 16x16 layout; three
// measured slower again), 3M complex products.  32 x 32 tiles for large batches; a 64 x 32
// tile moves 24 KB per K step for twice the products of a 32 x 32 tile's 16 KB.
// P[kz * n^2 + i + j n] = the split kz's products (raw, no scaling).
template <int GM, int GN>
__global__ void __launch_bounds__(256) gram_kernel(const ZBatch* __restrict__ zb, double2* __restrict__ P) {
    constexpr int TM = GM / 32, TN = GN / 32;   // 16x16 blocks per wave (2 x 2 waves)
    constexpr int NA = GM * ZBK / 256, NB = GN * ZBK / 256;
    __shared__ double2 As[2][ZBK][GM + 1];
    __shared__ double2 Bs[2][ZBK][GN + 1];
    // every tile of one Gram product on one XCD
    const long w = xcd_grouped(blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z),
                               (long)gridDim.x * gridDim.y * gridDim.z);
    const int bx = (int)(w % gridDim.x);
    const long rr = w / gridDim.x;
    const int kz = (int)(rr % gridDim.y), bz = (int)(rr / gridDim.y);
    const ZBatch e = zb[bz];
    const int n = e.n, K = e.k;
    const int mtiles = (n + GM - 1) / GM, ntiles = (n + GN - 1) / GN;
    if (bx >= mtiles * ntiles) return;
    const int mt = bx % mtiles, nt = bx / mtiles;
    const int m0 = mt * GM, n0 = nt * GN;
    if (m0 + GM <= n0) return;   // above the diagonal
    const double2* __restrict__ A = e.A;
    P += e.poff + (long)kz * n * n;
    const int kb = kz * e.kchunk, ke = min(K, kb + e.kchunk);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    d4 c1[TM][TN], c2[TM][TN], c3[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) c1[i][j] = c2[i][j] = c3[i][j] = d4{0, 0, 0, 0};
    // thread element idx: k-offset idx % 16 (16 consecutive rows of A, 256 bytes), column idx / 16
    struct Stage {
        double2 a[NA], b[NB];
    };
    auto gload = [&](int k0, Stage& g) {
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            const int idx = tid + v * 256, kk = idx % ZBK, i = idx / ZBK;
            const int gi = m0 + i, gk = k0 + kk;
            double2 a = (gi < n && gk < ke) ? A[gk + (long)gi * K] : make_double2(0.0, 0.0);
            a.y = -a.y;   // rows of A^*
            g.a[v] = a;
        }
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            const int idx = tid + v * 256, kk = idx % ZBK, j = idx / ZBK;
            const int gj = n0 + j, gk = k0 + kk;
            g.b[v] = (gj < n && gk < ke) ? A[gk + (long)gj * K] : make_double2(0.0, 0.0);
        }
    };
    auto lstore = [&](int buf, const Stage& g) {
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            const int idx = tid + v * 256;
            As[buf][idx % ZBK][idx / ZBK] = g.a[v];
        }
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            const int idx = tid + v * 256;
            Bs[buf][idx % ZBK][idx / ZBK] = g.b[v];
        }
    };
    auto step = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < ZBK / 4; ++kk) {
            double ar[TM], ai[TM], br[TN], bi[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const double2 a = As[buf][kk * 4 + lk][wm * (GM / 2) + i * 16 + lr];
                ar[i] = a.x;
                ai[i] = a.y;
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const double2 b = Bs[buf][kk * 4 + lk][wn * (GN / 2) + j * 16 + lr];
                br[j] = b.x;
                bi[j] = b.y;
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    c1[i][j] = mfma64(ar[i], br[j], c1[i][j]);
                    c2[i][j] = mfma64(ai[i], bi[j], c2[i][j]);
                    c3[i][j] = mfma64(ar[i] + ai[i], br[j] + bi[j], c3[i][j]);
                }
        }
    };
    // two K steps of global loads in flight while one is multiplied: register stages X and Y
    // alternate (the loop body is written twice so that each stage stays in its own registers)
    Stage X, Y;
    if (kb < ke) gload(kb, X);
    if (kb + ZBK < ke) gload(kb + ZBK, Y);
    if (kb < ke) lstore(0, X);
    __syncthreads();
    for (int k0 = kb; k0 < ke;) {
        if (k0 + 2 * ZBK < ke) gload(k0 + 2 * ZBK, X);
        step(0);
        if (k0 + ZBK < ke) lstore(1, Y);
        __syncthreads();
        k0 += ZBK;
        if (k0 >= ke) break;
        if (k0 + 2 * ZBK < ke) gload(k0 + 2 * ZBK, Y);
        step(1);
        if (k0 + ZBK < ke) lstore(0, X);
        __syncthreads();
        k0 += ZBK;
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = m0 + wm * (GM / 2) + i * 16 + lk + 4 * r;   // f64 MFMA D rows: (lane>>4) + 4r
                const int gj = n0 + wn * (GN / 2) + j * 16 + lr;
                if (gi >= n || gj >= n) continue;
                P[gi + (long)gj * n] = make_double2(c1[i][j][r] - c2[i][j][r], c3[i][j][r] - c1[i][j][r] - c2[i][j][r]);
            }
}

__global__ void zgemm_reduce_kernel(int M, int N, int nsplit, const double2* __restrict__ P, long pstride,
                                    double2* __restrict__ C, int ldc, double2 alpha, double2 beta, int tri, int tile) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= M) return;
    if (tri == 1 && (i / tile + 1) * tile <= (j / tile) * tile) return;
    {
        const long t = i + (long)j * M;
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

// 1/d to full FP64 precision: hardware reciprocal estimate refined by two
// Newton steps (each doubles the correct bits), cheaper in latency than the
// IEEE division sequence
__device__ inline double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// Registers of lane (r, g) = (lane & 15, lane >> 4) in the elimination of a 16x16 diagonal
// sub-block: the whole Hermitian block, M(r, 4g + q) for q < 4.
struct ElimRegs {
    double mr[4], mi[4];     // M(r, 4g + q)
    double lr0[4], li0[4];   // L_ss(r, 4g + q) before scaling: column 4g + q just before its step
    unsigned badm;           // bit K: pivot d_K not positive (replaced by 1)
};

__device__ inline double readlane64(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}

// x of lane 16 (lane >> 4) + K, in every lane of that 16-lane row (DPP row broadcast)
template <int K>
__device__ inline double bcast_row16(double x) {
    return __builtin_amdgcn_mov_dpp(x, 0x150 + K, 0xF, 0xF, false);   // one 64-bit DPP move
}

// Step K of the unscaled elimination of [D | I] (pivot d_K, Lt(i,K) = M(i,K)/d_K for the rows
// i > K, M(i,j) -= Lt(i,K) v_j with v_j = M(K,j) for j != K, which is X(K,j) left of the pivot
// and conj(M(j,K)) right of it, and v_K = d_K + 1, which turns column K into -Lt(.,K)).  All
// operands come from registers: the pivot by a lane read, M(r,K) by a lane shuffle from column
// group K >> 2, row K by a DPP broadcast from lane K of the lane's own 16-lane row.
template <int K>
__device__ __attribute__((always_inline)) inline void elim_step(ElimRegs& e, int r, int g) {
    constexpr int kk = K & 3, k4 = K >> 2;
    const double d = readlane64(e.mr[kk], K + 16 * k4);
    const bool ok = d > 0.0;
    e.badm |= ok ? 0u : 1u << K;
    const double dd = ok ? d : 1.0;
    e.lr0[kk] = g == k4 ? e.mr[kk] : e.lr0[kk];
    e.li0[kk] = g == k4 ? e.mi[kk] : e.li0[kk];
    if constexpr (K < 15) {   // no row lies below the last pivot
        const double cr = __shfl(e.mr[kk], r + 16 * k4), ci = __shfl(e.mi[kk], r + 16 * k4);
        double wr[4], wi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            wr[q] = bcast_row16<K>(e.mr[q]);
            wi[q] = bcast_row16<K>(e.mi[q]);
        }
        wr[kk] = g == k4 ? dd + 1.0 : wr[kk];
        wi[kk] = g == k4 ? 0.0 : wi[kk];
        // 1/d_K = r0 (1 + eps) to full precision (one Newton step on the estimate r0)
        const double r0 = __builtin_amdgcn_rcp(dd);
        const double eps = fma(-dd, r0, 1.0);
        const double tr = cr * r0, ti = ci * r0;
        const bool live = r > K;
        const double lr = live ? fma(tr, eps, tr) : 0.0, li = live ? fma(ti, eps, ti) : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double xr = e.mr[q], xi = e.mi[q];
            e.mr[q] = fma(-lr, wr[q], fma(li, wi[q], xr));
            e.mi[q] = fma(-lr, wi[q], fma(-li, wr[q], xi));
        }
    }
}

template <int K>
__device__ __attribute__((always_inline)) inline void elim_steps(ElimRegs& e, int r, int g) {
    elim_step<K>(e, r, g);
    if constexpr (K + 1 < 16) elim_steps<K + 1>(e, r, g);
}

// LDS of one diagonal-block factorisation (rows padded to 65 entries)
struct CholLds {
    double2 S[64][65];     // Schur complement -> L (row-major, lower part)
    double2 Z[64][65];     // inverse accumulation -> L^{-1} (row-major, lower part, zero upper part)
    double cs[64];         // 1/sqrt of the pivots: column scales of the diagonal 16x16 blocks of L
};

// C(16x16 tile) = sum_{k<16} A(i, k) B(k, c) on the matrix cores, A(i, k) = a(i, k) and
// B(k, c) = b(k, c) read through the functors.  Computed transposed, C^T = B^T A^T, so that lane
// (i, g) = (lane & 15, lane >> 4) ends with C(i, g + 4 q) in element q of cr / ci: the A operand
// is B^T (lane (c, kq) holds B(4t + kq, c)), the B operand A^T (lane (kq, i) holds A(i, 4t + kq)).
// Two LDS reads per lane and k-step of 4 (the vector form needs five per k); four independent
// accumulation chains.
template <class FA, class FB>
__device__ inline void tile16_load(double2 (&x)[4], double2 (&y)[4], FA a, FB b) {
    const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        x[t] = a(i, 4 * t + kq);
        y[t] = b(4 * t + kq, i);
    }
}
__device__ inline void tile16_prod(const double2 (&x)[4], const double2 (&y)[4], d4& cr, d4& ci) {
    d4 r1 = {0, 0, 0, 0}, r2 = {0, 0, 0, 0}, i1 = {0, 0, 0, 0}, i2 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        r1 = mfma64(y[t].x, x[t].x, r1);
        r2 = mfma64(y[t].y, x[t].y, r2);
        i1 = mfma64(y[t].x, x[t].y, i1);
        i2 = mfma64(y[t].y, x[t].x, i2);
    }
    cr = r1 - r2;
    ci = i1 + i2;
}
template <class FA, class FB>
__device__ inline void tile16_mfma(d4& cr, d4& ci, FA a, FB b) {
    double2 x[4], y[4];
    tile16_load(x, y, a, b);
    tile16_prod(x, y, cr, ci);
}

// One update tile of the factorisation's trailing step (rows padded to 65 entries):
// O(i, c) -= sum_k A(i, k) B(k, c), A(i, k) = A[65 i + k], B(k, c) = B[sk k + sc c] conjugated
// when cs = -1, O(i, c) = O[65 i + c].
struct TileRef {
    const double2* A;
    const double2* B;
    double2* O;
    int sk, sc;
    double cs;
};

// Cholesky factor and inverse of one Hermitian positive definite diagonal
// block of order nb <= 64, by a workgroup of exactly 256 threads: G (lower
// triangle read, ld ldg) + shift I = L L^*.  On return (after a barrier) s.Z
// holds L^{-1} row-major with zero upper triangle and s.S holds L in its lower
// triangle (orders below 64 padded with the identity), except that the strict
// lower parts of its diagonal 16x16 blocks lack their column scales s.cs; if
// Lout / Zout are set, L and L^{-1} are written there (lower triangles, ld ldl / ldz).
// Returns the 1-based index of the first non-positive pivot (0 if none), the
// same in every thread.
//
// Recursive blocking by 16 columns.  Sub-block s (rows/columns b0..b0+15):
//  F  one wavefront factors the 16x16 diagonal block D = L_ss L_ss^* and its
//     inverse by unscaled elimination of [D | I] (step k: pivot d_k, Lt(i,k) =
//     D(i,k)/d_k, M(i,j) -= Lt(i,k) v_j over one array M holding D right of the
//     eliminated columns and the unit factor's inverse X left of them, v_j =
//     conj(D(j,k)) for j > k, X(k,j) for j < k, d_k + 1 for j = k), entirely in
//     registers: each lane holds four entries of the whole Hermitian block, so
//     v_j is row k's entry (a DPP row broadcast) and the multipliers' column
//     comes from one of the four 16-lane rows (a lane shuffle);
//  P  L(i,s) = S(i,s) L_ss^{-*} for the rows below, and Z(s,j) = L_ss^{-1} W(s,j)
//     for the columns left of the block, W(s,j) = -sum_{l<s} L(s,l) Z(l,j) being
//     what Z holds there;
//  U  S(i,j) -= L(i,s) L(j,s)^* (trailing, lower) and W(i,j) -= L(i,s) Z(s,j)
//     for the rows below (j up to the block, Z(s,s) = L_ss^{-1}).
// P and U work on 16x16 tiles spread over the 4 wavefronts, on the matrix cores.
__device__ __attribute__((always_inline)) int chol64_lds(const double2* __restrict__ G, int ldg, int nb, double shift, CholLds& s,
                          double2* __restrict__ Lout, int ldl, double2* __restrict__ Zout, int ldz) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;   // tile row, column group (columns 4g..4g+3)
    // the shifted lower triangle (j <= i), padded with the identity beyond order nb, and zero where
    // `use` is false; the load itself is unconditional (an entry outside reads G[0], nb >= 1), so
    // that a thread's loads are all in flight before the first wait
    auto gval = [&](int i, int j, bool use) {
        const bool in = use && i < nb;
        const double2 x = G[in ? i + (long)j * ldg : 0];
        const double2 v = in ? x : make_double2(0.0, 0.0);
        return !use || i != j ? v : i < nb ? make_double2(v.x + shift, v.y) : make_double2(1.0, 0.0);
    };
    // wavefront 0 takes its entries of the first diagonal 16x16 block straight from memory (the
    // whole Hermitian block) and starts eliminating while the others bring the rest into LDS
    double2 m0[4];
    if (wave == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * g + q;
            const double2 v = gval(c <= r ? r : c, c <= r ? c : r, true);
            m0[q] = make_double2(v.x, c <= r ? v.y : -v.y);
        }
    }
    // L(i, j), the diagonal blocks' column scales applied
    auto lval = [&](int i, int j) {
        const double2 v = s.S[i][j];
        const double c = ((i >> 4) == (j >> 4) && i != j) ? s.cs[j] : 1.0;
        return make_double2(v.x * c, v.y * c);
    };
    // L's column block cb and Z's row block cb to memory by threads t0.. (nt of them): final once
    // sub-block cb's panel step is done (later steps touch only columns / rows beyond it)
    auto write_block = [&](int cb, int t, int nt) {
        const int c0 = 16 * cb;
        if (Lout)   // rows c0..63 as 16x16 tiles; consecutive threads: consecutive rows of a column
#pragma unroll 4
            for (int e = t; e < 256 * (4 - cb); e += nt) {
                const int i = c0 + 16 * (e >> 8) + (e & 15), j = c0 + ((e >> 4) & 15);
                if (i < nb && j <= i) Lout[i + (long)j * ldl] = lval(i, j);
            }
        if (Zout)
#pragma unroll 4
            for (int e = t; e < 16 * (c0 + 16); e += nt) {
                const int i = c0 + (e & 15), j = e >> 4;
                if (i < nb && j <= i) Zout[i + (long)j * ldz] = s.Z[i][j];
            }
    };
    int bad = 0;
    for (int sb = 0; sb < 4; ++sb) {
        const int b0 = 16 * sb;
        // ---- F: 16x16 diagonal block by wavefront 0 (lane (r, g) holds M(r, 4g + q), q < 4; the
        //      whole Hermitian block, so that row k supplies the conjugated column below the pivot)
        if (wave == 0) {
            ElimRegs e;
            e.badm = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = 4 * g + q;
                double2 v = m0[q];
                if (sb > 0) {
                    v = (c <= r) ? s.S[b0 + r][b0 + c] : s.S[b0 + c][b0 + r];
                    v.y = c <= r ? v.y : -v.y;
                }
                e.mr[q] = v.x;
                e.mi[q] = v.y;
                e.lr0[q] = e.li0[q] = 0.0;
            }
            elim_steps<0>(e, r, g);
            if (bad == 0 && e.badm) bad = b0 + __builtin_ctz(e.badm) + 1;
            // d_r: M(r, r) is left as it was at its own step, in register r & 3 of lane (r, r >> 2)
            double dr = e.mr[0];
#pragma unroll
            for (int q = 1; q < 4; ++q) dr = (r & 3) == q ? e.mr[q] : dr;
            dr = __shfl(dr, r + 16 * (r >> 2));
            const double pr = dr > 0.0 ? dr : 1.0;
            // L_ss^{-1} into Z (lower part; upper part of the Z block stays zero), L_ss into S with
            // its strict lower part unscaled (column c is scaled by 1/sqrt(d_c) on the way out)
            const double sdr = sqrt(pr), rdr = recip(sdr);
            if (g == 0) s.cs[b0 + r] = rdr;
            // every entry of the lane is written (no branches): the upper part of the Z block must
            // stay zero, the upper part of the S block is never read
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = 4 * g + q;
                const bool lo = c < r, dg = c == r;
                s.S[b0 + r][b0 + c] = make_double2(dg ? sdr : e.lr0[q], dg ? 0.0 : e.li0[q]);
                s.Z[b0 + r][b0 + c] = make_double2(lo ? e.mr[q] * rdr : dg ? rdr : 0.0, lo ? e.mi[q] * rdr : 0.0);
            }
        } else if (sb == 0) {
            // the rest of the block into LDS (S and Z but their first diagonal 16x16 blocks, which
            // wavefront 0 writes after its elimination), every load issued before the first wait
            constexpr int NT = 192, NU = (64 * 64 + NT - 1) / NT;
            double2 v[NU];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int e = tid - 64 + NT * u, i = e & 63, j = e >> 6;   // consecutive rows of a column
                v[u] = gval(i, j, e < 64 * 64 && j <= i && i >= 16);
            }
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int e = tid - 64 + NT * u, i = e & 63, j = e >> 6;
                if (e < 64 * 64 && (i >= 16 || j >= 16)) {
                    s.S[i][j] = v[u];
                    s.Z[i][j] = make_double2(0.0, 0.0);
                }
            }
        } else {
            write_block(sb - 1, tid - 64, blockDim.x - 64);   // while wavefront 0 eliminates
        }
        __syncthreads();
        // ---- P: panel below (tiles it = sb+1..3) and Z row block (tiles jt = 0..sb-1), into registers
        const int np = 3 - sb, ntp = np + sb;
        d4 pr_ = {0, 0, 0, 0}, pi_ = {0, 0, 0, 0};
        int pt = -1;
        for (int t = wave; t < ntp; t += 4) pt = t;   // each wavefront owns at most one tile (ntp <= 3)
        if (pt >= 0) {
            if (pt < np) {
                const int i0 = b0 + 16 * (pt + 1);
                tile16_mfma(pr_, pi_, [&](int i, int k) { return s.S[i0 + i][b0 + k]; },
                            [&](int k, int c) { const double2 z = s.Z[b0 + c][b0 + k];
                                                return make_double2(z.x, -z.y); });
            } else {
                const int j0 = 16 * (pt - np);
                tile16_mfma(pr_, pi_, [&](int i, int k) { return s.Z[b0 + i][b0 + k]; },
                            [&](int k, int c) { return s.Z[b0 + k][j0 + c]; });
            }
        }
        __syncthreads();
        if (pt >= 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (pt < np) s.S[b0 + 16 * (pt + 1) + r][b0 + g + 4 * q] = make_double2(pr_[q], pi_[q]);
                else s.Z[b0 + r][16 * (pt - np) + g + 4 * q] = make_double2(pr_[q], pi_[q]);
            }
        }
        __syncthreads();
        // ---- U: trailing lower tiles (sb < jt <= it) and W tiles (it > sb, jt <= sb), a
        //      wavefront's tiles t = wave + 4u in turn, each tile's operands loaded while the
        //      previous one is on the matrix cores (no tile reads what another one writes)
        const int ntr = np * (np + 1) / 2, ntot = ntr + np * (sb + 1);
        auto tile_ref = [&](int t) {
            TileRef f;
            if (t < ntr) {
                int a = 0;
                while ((a + 1) * (a + 2) / 2 <= t) ++a;
                const int it = sb + 1 + a, jt = sb + 1 + (t - a * (a + 1) / 2);
                f = TileRef{&s.S[16 * it][b0], &s.S[16 * jt][b0], &s.S[16 * it][16 * jt], 1, 65, -1.0};
            } else {
                const int u = t - ntr, it = sb + 1 + u % np, jt = u / np;
                f = TileRef{&s.S[16 * it][b0], &s.Z[b0][16 * jt], &s.Z[16 * it][16 * jt], 65, 1, 1.0};
            }
            return f;
        };
        auto ops = [&](const TileRef& f, double2 (&x)[4], double2 (&y)[4]) {
            tile16_load(x, y, [&](int i, int k) { return f.A[65 * i + k]; },
                        [&](int k, int c) { const double2 v = f.B[f.sk * k + f.sc * c];
                                            return make_double2(v.x, f.cs * v.y); });
        };
        if (wave < ntot) {
            int t = wave;
            TileRef f = tile_ref(t);
            double2 x[4], y[4];
            ops(f, x, y);
            while (true) {
                const int tn = t + 4;
                TileRef fn = f;
                double2 xn[4], yn[4];
                if (tn < ntot) {
                    fn = tile_ref(tn);
                    ops(fn, xn, yn);
                }
                d4 cr, ci;
                tile16_prod(x, y, cr, ci);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double2& o = f.O[65 * r + g + 4 * q];
                    o.x -= cr[q];
                    o.y -= ci[q];
                }
                if (tn >= ntot) break;
                t = tn;
                f = fn;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    x[u] = xn[u];
                    y[u] = yn[u];
                }
            }
        }
        __syncthreads();
    }
    // the first failure (wavefront 0 saw every pivot), the same in every thread
    __shared__ int bad_s;
    if (tid == 0) bad_s = bad;
    __syncthreads();
    const int first = bad_s;
    write_block(3, tid, blockDim.x);
    return first;
}

// Block step of the blocked Cholesky factorisation and inverse of an order-nc
// Hermitian positive definite matrix (G, lower triangle, ld nc).  The step's
// columns kb..r0-1 (r0 = kb + sp.wtot) form nq diagonal sub-blocks q,
// columns kb + off[q] .. kb + off[q+1] - 1 (at most 64 each), that do not
// couple (G vanishes between them, so L and L^{-1} do too): each is factored
// on its own.  Z = L^{-1} is built block row by block row: W(i,j) accumulates
// -sum_l L(i,l) Z(l,j) over the eliminated columns l, and Z(q,j) = Z(q,q) W(q,j)
// once block row q's W is complete.  Two launches per step before the update:
//   diagonal: one workgroup per sub-block factors it in LDS and writes L(q,q),
//     Z(q,q) = L(q,q)^{-1} (lower triangles; the upper ones stay zero) and the
//     first breakdown to *info;
//   slabs: one workgroup per 32-row slab of the rows r0..nc-1, L(i,q) =
//     G(i,q) Z(q,q)^*, and per 32-column slab j0 < kb of block row q of Z,
//     Z(q,j) = Z(q,q) W(q,j); Z(q,q) is read from memory (an L2-resident 64 KB
//     block shared by the step's workgroups), so a slab workgroup needs no
//     refactorisation and little LDS, and many fit on a CU.
__device__ __attribute__((always_inline)) inline void chol_diag_body(const double2* __restrict__ G, int nc, int kq, int nbq, double shift,
                                      double2* __restrict__ L, double2* __restrict__ Z, int* info, CholLds& s) {
    if (nbq <= 0) return;   // an empty block (the factorisation reads element (kq, kq) unconditionally)
    const long dk = kq + (long)kq * nc;
    const int bad = chol64_lds(G + dk, nc, nbq, shift, s, L + dk, nc, Z + dk, nc);
    if (threadIdx.x == 0 && bad && info) atomicCAS(info, 0, kq + bad);
}

// Z(q,q)(r, k) of the sub-block at kq of order nbq (lower triangle; zero outside the block)
__device__ inline double2 zqq_at(const double2* Z, int nc, int kq, int nbq, int r, int k) {
    return (r < nbq && k <= r) ? Z[kq + r + (long)(kq + k) * nc] : make_double2(0.0, 0.0);
}

// slab role of one sub-block (kq, nbq) of the step with trailing rows from r0: roles
// 0..np-1 are row slabs of L, the rest column slabs of block row q of Z
__device__ __attribute__((always_inline)) inline void chol_slab_body(const double2* __restrict__ G, int nc, int kb, int r0, int kq, int nbq,
                                      double2* __restrict__ L, double2* Z, const double2* __restrict__ W, int np,
                                      int role) {
    const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63, lr = ln & 15, lk = ln >> 4;
    if (role < np) {
        // L(i,c) = sum_k G(i,k) conj(Z(c,k)) on the matrix cores for the rows i0..i0+31: 32 x 64 as
        // 2 x 4 tiles of 16 x 16, two per wavefront (tile row wave >> 1, tile columns 2 (wave & 1) +
        // {0, 1}); A operand lane (row lane & 15, k lane >> 4), B operand lane (k lane >> 4, column
        // lane & 15), result rows (lane >> 4) + 4 r of each tile.  Both operands straight from memory
        // (16 consecutive rows of one column per load), four k-steps in flight.
        const int i0 = r0 + 32 * role, ti = wv >> 1, i = i0 + 16 * ti + lr;
        const int cb = 32 * (wv & 1);
        d4 cr[2], ci[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) { cr[t] = d4{0, 0, 0, 0}; ci[t] = d4{0, 0, 0, 0}; }
        auto load = [&](int k0, double2* a, double2 (*z)[2]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + 4 * u + lk;
                a[u] = (i < nc && k < nbq) ? G[i + (long)(kq + k) * nc] : make_double2(0.0, 0.0);
#pragma unroll
                for (int t = 0; t < 2; ++t) z[u][t] = zqq_at(Z, nc, kq, nbq, cb + 16 * t + lr, k);
            }
        };
        double2 a[4], z[4][2], na[4], nz[4][2];
        load(0, a, z);
#pragma unroll
        for (int k0 = 0; k0 < 64; k0 += 16) {
            if (k0 + 16 < 64) load(k0 + 16, na, nz);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < 2; ++t) {   // B = conj(Z)^T
                    cr[t] = mfma64(a[u].x, z[u][t].x, cr[t]);
                    cr[t] = mfma64(a[u].y, z[u][t].y, cr[t]);
                    ci[t] = mfma64(-a[u].x, z[u][t].y, ci[t]);
                    ci[t] = mfma64(a[u].y, z[u][t].x, ci[t]);
                }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = na[u];
#pragma unroll
                for (int t = 0; t < 2; ++t) z[u][t] = nz[u][t];
            }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int io = i0 + 16 * ti + lk + 4 * r, c = cb + 16 * t + lr;
                if (io < nc && c < nbq) L[io + (long)(kq + c) * nc] = make_double2(cr[t][r], ci[t][r]);
            }
        return;
    }
    // columns j0..j0+31 (< kb) of block row q of Z: Sw[k][c] = W(kq + k, j0 + c), staged in LDS by
    // coalesced loads (consecutive threads: consecutive k of one column)
    __shared__ double2 Sw[64][33];
    const int j0 = 32 * (role - np);
    {
        double2 v[8];   // every load issued before the first wait
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u, k = e & 63, c = e >> 6;
            v[u] = (k < nbq && j0 + c < kb) ? W[kq + k + (long)(j0 + c) * nc] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            Sw[e & 63][e >> 6] = v[u];
        }
    }
    __syncthreads();
    // Z(q, j) = Z(q,q) W(q, j) on the matrix cores: 64 x 32 as 4 x 2 tiles of 16 x 16, two per
    // wavefront (tile rows 2 (wave >> 1) + {0, 1}, tile column wave & 1); A operand Z(q,q) from memory
    const int tj = wv & 1, rb = 32 * (wv >> 1);
    d4 cr[2], ci[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) { cr[t] = d4{0, 0, 0, 0}; ci[t] = d4{0, 0, 0, 0}; }
    auto loadz = [&](int k0, double2 (*z)[2]) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 2; ++t) z[u][t] = zqq_at(Z, nc, kq, nbq, rb + 16 * t + lr, k0 + 4 * u + lk);
    };
    double2 z[4][2], nzq[4][2];
    loadz(0, z);
#pragma unroll
    for (int k0 = 0; k0 < 64; k0 += 16) {
        if (k0 + 16 < 64) loadz(k0 + 16, nzq);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double2 w = Sw[k0 + 4 * u + lk][16 * tj + lr];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                cr[t] = mfma64(z[u][t].x, w.x, cr[t]);
                cr[t] = mfma64(-z[u][t].y, w.y, cr[t]);
                ci[t] = mfma64(z[u][t].x, w.y, ci[t]);
                ci[t] = mfma64(z[u][t].y, w.x, ci[t]);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 2; ++t) z[u][t] = nzq[u][t];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rr = rb + 16 * t + lk + 4 * r, j = j0 + 16 * tj + lr;
            if (rr < nbq && j < kb) Z[kq + rr + (long)j * nc] = make_double2(cr[t][r], ci[t][r]);
        }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
chol_diag_kernel(const double2* __restrict__ G, int nc, CholStepDev sp, double shift, double2* __restrict__ L,
                 double2* __restrict__ Z, int* info) {
    __shared__ CholLds s;
    const int q = blockIdx.x;
    chol_diag_body(G, nc, sp.kb + sp.off[q], sp.off[q + 1] - sp.off[q], shift, L, Z, info, s);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
chol_slab_kernel(const double2* __restrict__ G, int nc, CholStepDev sp, double2* __restrict__ L, double2* Z,
                 const double2* __restrict__ W, int np, int nz) {
    const int roles = np + nz;
    const int q = blockIdx.x / roles, role = blockIdx.x - q * roles;
    const int kq = sp.kb + sp.off[q], nbq = sp.off[q + 1] - sp.off[q];
    chol_slab_body(G, nc, sp.kb, sp.kb + sp.wtot, kq, nbq, L, Z, W, np, role);
}

// One Cholesky step of several matrices at once (the fronts of one elimination-tree
// height): entry blockIdx.x (diagonal) or blockIdx.y (slabs) factors its sub-block
// kb..kb+w-1; slab workgroups past the entry's roles exit.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
chol_diag_batched_kernel(const CholBatchEntry* __restrict__ ent, int* info) {
    __shared__ CholLds s;
    const CholBatchEntry e = ent[blockIdx.x];
    chol_diag_body(e.G, e.nc, e.kb, e.w, 0.0, e.L, e.Z, info, s);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
chol_slab_batched_kernel(const CholBatchEntry* __restrict__ ent) {
    const CholBatchEntry e = ent[blockIdx.y];
    if ((int)blockIdx.x >= e.np + e.nz) return;
    chol_slab_body(e.G, e.nc, e.kb, e.kb + e.w, e.kb, e.w, e.L, e.Z, e.W, e.np, blockIdx.x);
}

// Update after the block step kb..r0-1 (r0 = kb + wtot): 64 x 64 tiles of
//   the trailing Schur complement  G(i,j) -= sum_k L(i,k) conj(L(j,k)),  r0 <= j <= i (tile-wise lower),
//   the inverse accumulation       W(i,j) -= sum_k L(i,k) Z(k,j),        i >= r0, j < r0,
// k over the step's columns (for j in the step, Z(k,j) is the step's own block-diagonal
// inverse and W starts from zero).  Computed transposed on the matrix cores,
// C^T(j,i) = sum_k B(k,j) L(i,k) with B(k,j) = conj(L(j,k)) or Z(k,j): the result lanes
// then hold consecutive rows i of a column j, so the read-modify-write of C is
// coalesced, and both operands come straight from memory (16 consecutive rows of one
// column per load; Z(k,j): 4 consecutive k of 16 columns), no LDS.  Four wavefronts, each
// a 32 x 32 quarter of the tile as 2 x 2 blocks of 16 x 16, two k-steps of loads in flight.
__device__ __attribute__((always_inline)) inline void chol_update64_body(double2* __restrict__ G, int nc, int kb,
                                                                       int wtot, const double2* __restrict__ L,
                                                                       const double2* __restrict__ Z,
                                                                       double2* __restrict__ W, int bx) {
    constexpr int BW = 2, TILE = 64;
    const int r0 = kb + wtot, tid = threadIdx.x;
    const int ntr = (nc - r0 + TILE - 1) / TILE;
    int t = bx, i0, j0;
    bool trail;
    const int ntri = ntr * (ntr + 1) / 2;
    if (t < ntri) {
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= t) ++a;
        i0 = r0 + TILE * a;
        j0 = r0 + TILE * (t - a * (a + 1) / 2);
        trail = true;
    } else {
        t -= ntri;
        i0 = r0 + TILE * (t % ntr);
        j0 = TILE * (t / ntr);
        trail = false;
    }
    const int wv = tid >> 6, ln = tid & 63, lr = ln & 15, lk = ln >> 4;
    const int ib = i0 + 16 * BW * (wv & 1), jb = j0 + 16 * BW * (wv >> 1);
    d4 c1[BW][BW], c2[BW][BW], c3[BW][BW];   // 3M products: ar br, ai bi, (ar + ai)(br + bi)
#pragma unroll
    for (int x = 0; x < BW; ++x)
#pragma unroll
        for (int y = 0; y < BW; ++y) { c1[x][y] = c2[x][y] = c3[x][y] = d4{0, 0, 0, 0}; }
    // operands of k-step ks (k = 4 ks + lane >> 4): A' (row j = jb + 16 tj + lane & 15),
    // B' (column i = ib + 16 ti + lane & 15)
    auto load = [&](int ks, double2* av, double2* bv) {
        const int k = 4 * ks + lk;
        const bool kin = k < wtot;
#pragma unroll
        for (int x = 0; x < BW; ++x) {
            const int j = jb + 16 * x + lr, i = ib + 16 * x + lr;
            if (trail) {
                const double2 v = (kin && j < nc) ? L[j + (long)(kb + k) * nc] : make_double2(0.0, 0.0);
                av[x] = make_double2(v.x, -v.y);
            } else {
                av[x] = (kin && j < r0) ? Z[kb + k + (long)j * nc] : make_double2(0.0, 0.0);
            }
            bv[x] = (kin && i < nc) ? L[i + (long)(kb + k) * nc] : make_double2(0.0, 0.0);
        }
    };
    // stages of S k-steps, the next stage's loads in flight (one: with the three 3M accumulators a
    // second stage needs more registers than three wavefronts per SIMD leave, measured slower)
    constexpr int S = 1;
    const int nks = (wtot + 3) / 4;
    double2 a[S][BW], b[S][BW], na[S][BW], nb[S][BW];
#pragma unroll
    for (int u = 0; u < S; ++u) load(u, a[u], b[u]);
    for (int ks = 0; ks < nks; ks += S) {
        if (ks + S < nks) {
#pragma unroll
            for (int u = 0; u < S; ++u) load(ks + S + u, na[u], nb[u]);
        }
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
            for (int x = 0; x < BW; ++x)
#pragma unroll
                for (int y = 0; y < BW; ++y) {   // D'(j, i) += A'(j, k) B'(k, i), complex
                    c1[x][y] = mfma64(a[u][x].x, b[u][y].x, c1[x][y]);
                    c2[x][y] = mfma64(a[u][x].y, b[u][y].y, c2[x][y]);
                    c3[x][y] = mfma64(a[u][x].x + a[u][x].y, b[u][y].x + b[u][y].y, c3[x][y]);
                }
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
            for (int x = 0; x < BW; ++x) { a[u][x] = na[u][x]; b[u][x] = nb[u][x]; }
    }
    // result lane: rows j = jb + 16 x + (lane >> 4) + 4 r, column i = ib + 16 y + lane & 15
    double2* C = trail ? G : W;
#pragma unroll
    for (int x = 0; x < BW; ++x)
#pragma unroll
        for (int y = 0; y < BW; ++y) {
            const int i = ib + 16 * y + lr;
            bool ok[4];
            double2 cv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {   // every load before the first wait
                const int j = jb + 16 * x + lk + 4 * r;
                ok[r] = i < nc && (trail ? (j < nc && j <= i) : j < r0);
                cv[r] = ok[r] ? C[i + (long)j * nc] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jb + 16 * x + lk + 4 * r;
                const double pr = c1[x][y][r] - c2[x][y][r], pi = c3[x][y][r] - c1[x][y][r] - c2[x][y][r];
                if (ok[r]) C[i + (long)j * nc] = make_double2(cv[r].x - pr, cv[r].y - pi);
            }
        }
}


// The same update in 32 x 32 tiles (small matrices: four times the workgroups) of
//   the trailing Schur complement  G(i,j) -= sum_k L(i,k) conj(L(j,k)),  r0 <= j <= i (tile-wise lower),
//   the inverse accumulation       W(i,j) -= sum_k L(i,k) Z(k,j),        i >= r0, j < r0,
// k over the step's columns in chunks of 64 (for j in the step, Z(k,j) is the
// step's own block-diagonal inverse and W starts from zero).  Both operands
// staged in LDS; 2 x 2 entries per thread.
__device__ __attribute__((always_inline)) inline void chol_update32_body(double2* __restrict__ G, int nc, int kb, int wtot,
                                        const double2* __restrict__ L, const double2* __restrict__ Z,
                                        double2* __restrict__ W, int ntr, int bx) {
    __shared__ double2 A[64][33];   // A[k][r] = L(i0 + r, k0 + k)
    __shared__ double2 B[64][33];   // B[k][c] = conj(L(j0 + c, k0 + k)) or Z(k0 + k, j0 + c)
    const int r0 = kb + wtot, tid = threadIdx.x;
    int t = bx, i0, j0;
    bool trail;
    const int ntri = ntr * (ntr + 1) / 2;
    if (t < ntri) {
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= t) ++a;
        i0 = r0 + 32 * a;
        j0 = r0 + 32 * (t - a * (a + 1) / 2);
        trail = true;
    } else {
        t -= ntri;
        i0 = r0 + 32 * (t % ntr);
        j0 = 32 * (t / ntr);
        trail = false;
    }
    // the 32 x 32 tile on the matrix cores: one 16 x 16 quarter per wavefront (rows 16 (wave >> 1),
    // columns 16 (wave & 1)); A operand lane (row lane & 15, k lane >> 4), B operand lane (k lane >> 4,
    // column lane & 15), result rows (lane >> 4) + 4 r
    const int wv = tid >> 6, ln = tid & 63, lr = ln & 15, lk = ln >> 4;
    const int ti = wv >> 1, tj = wv & 1;
    d4 c1 = d4{0, 0, 0, 0}, c2 = c1, c3 = c1;   // 3M products: ar br, ai bi, (ar + ai)(br + bi)
    for (int k0 = kb; k0 < r0; k0 += 64) {
        const int kn = min(64, r0 - k0);
        // both operands' loads of the chunk issued before the first wait
        double2 av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u, k = e >> 5, r = e & 31;
            const int i = i0 + r, j = j0 + r;
            const bool kin = k < kn;
            av[u] = (kin && i < nc) ? L[i + (long)(k0 + k) * nc] : make_double2(0.0, 0.0);
            if (trail) {
                const double2 v = (kin && j < nc) ? L[j + (long)(k0 + k) * nc] : make_double2(0.0, 0.0);
                bv[u] = make_double2(v.x, -v.y);
            } else {
                bv[u] = (kin && j < r0) ? Z[k0 + k + (long)j * nc] : make_double2(0.0, 0.0);
            }
        }
        if (k0 > kb) __syncthreads();   // the previous chunk's operands are consumed
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u, k = e >> 5, r = e & 31;
            A[k][r] = av[u];
            B[k][r] = bv[u];
        }
        __syncthreads();
#pragma unroll 4
        for (int kk0 = 0; kk0 < 64; kk0 += 4) {
            const double2 a = A[kk0 + lk][16 * ti + lr], b = B[kk0 + lk][16 * tj + lr];
            c1 = mfma64(a.x, b.x, c1);
            c2 = mfma64(a.y, b.y, c2);
            c3 = mfma64(a.x + a.y, b.x + b.y, c3);
        }
    }
    double2* C = trail ? G : W;
    const int j = j0 + 16 * tj + lr;
    bool ok[4];
    double2 cv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {   // every load before the first wait
        const int i = i0 + 16 * ti + lk + 4 * r;
        ok[r] = i < nc && j < nc && !(trail && j > i) && !(!trail && j >= r0);
        cv[r] = ok[r] ? C[i + (long)j * nc] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * ti + lk + 4 * r;
        const double pr = c1[r] - c2[r], pi = c3[r] - c1[r] - c2[r];
        if (ok[r]) C[i + (long)j * nc] = make_double2(cv[r].x - pr, cv[r].y - pi);
    }
}


template <bool WIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WIDE ? 3 : 1)))
chol_update_kernel(double2* __restrict__ G, int nc, int kb, int wtot, const double2* __restrict__ L,
                   const double2* __restrict__ Z, double2* __restrict__ W) {
    if constexpr (WIDE) chol_update64_body(G, nc, kb, wtot, L, Z, W, blockIdx.x);
    else chol_update32_body(G, nc, kb, wtot, L, Z, W, (nc - kb - wtot + 31) / 32, blockIdx.x);
}

// The update of one step of several matrices at once (entry blockIdx.y; workgroups past
// the entry's tiles exit).
template <bool WIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WIDE ? 3 : 1)))
chol_update_batched_kernel(const CholBatchEntry* __restrict__ ent) {
    const CholBatchEntry e = ent[blockIdx.y];
    if ((int)blockIdx.x >= chol_update_tiles(e.nc, e.kb, e.w, WIDE ? 64 : 32)) return;
    if constexpr (WIDE) chol_update64_body(e.G, e.nc, e.kb, e.w, e.L, e.Z, e.W, blockIdx.x);
    else chol_update32_body(e.G, e.nc, e.kb, e.w, e.L, e.Z, e.W, e.np, blockIdx.x);
}

// max and min Cholesky pivot ratio estimate: diag of L (ld) -> out[0] = max |L_ii|^2, out[1] = min |L_ii|^2
__global__ void diag_range_kernel(const double2* __restrict__ L, int n, int ld, double* out) {
    __shared__ double mx[256], mn[256];
    double a = 0.0, b = 1e308;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double v = L[i + (long)i * ld].x;
        a = fmax(a, v * v);
        b = fmin(b, v * v);
    }
    mx[threadIdx.x] = a;
    mn[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
            mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = mx[0]; out[1] = mn[0]; }
}

// y = alpha op(A) x + beta y, op = conjugate transpose: one workgroup per output
// entry j (a length-m dot product of column j), A column-major m x n; lower: A is
// lower triangular, so column j starts at row j.
__global__ void __launch_bounds__(256)
zgemv_c_kernel(int m, const double2* __restrict__ A, int lda, const double2* __restrict__ x, double2* y,
               double2 alpha, double2 beta, int lower) {
    const int j = blockIdx.x;
    __shared__ double rr[256], ri[256];
    double sr = 0.0, si = 0.0;
    const double2* col = A + (long)j * lda;
    for (int i = (lower ? j : 0) + threadIdx.x; i < m; i += 256) {
        const double2 a = col[i], v = x[i];
        sr += a.x * v.x + a.y * v.y;
        si += a.x * v.y - a.y * v.x;
    }
    rr[threadIdx.x] = sr;
    ri[threadIdx.x] = si;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) { rr[threadIdx.x] += rr[threadIdx.x + w]; ri[threadIdx.x] += ri[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double2 o = make_double2(alpha.x * rr[0] - alpha.y * ri[0], alpha.x * ri[0] + alpha.y * rr[0]);
        if (beta.x != 0.0 || beta.y != 0.0) {
            const double2 c = y[j];
            o.x += beta.x * c.x - beta.y * c.y;
            o.y += beta.x * c.y + beta.y * c.x;
        }
        y[j] = o;
    }
}

// y += alpha A x (A column-major m x n): thread per row, 64-column chunks per
// workgroup, partial sums added atomically (y pre-scaled by beta separately).
__global__ void __launch_bounds__(256)
zgemv_n_kernel(int m, int n, const double2* __restrict__ A, int lda, const double2* __restrict__ x, double* y,
               double2 alpha) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j0 = blockIdx.y * 64;
    const int j1 = min(n, j0 + 64);
    if (i >= m) return;
    double sr = 0.0, si = 0.0;
    const double2* a = A + i;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
        const double2 av = a[(long)j * lda], v = x[j];
        sr += av.x * v.x - av.y * v.y;
        si += av.x * v.y + av.y * v.x;
    }
    atomicAdd(&y[2 * i], alpha.x * sr - alpha.y * si);
    atomicAdd(&y[2 * i + 1], alpha.x * si + alpha.y * sr);
}

// y = alpha A x (A column-major m x n, y overwritten); lower: A is lower triangular
// (row i reads columns j <= i only).  16 rows x 16 column groups per workgroup; the
// groups' partial sums are added in a fixed order (no atomics).
__global__ void __launch_bounds__(256)
zgemv_n_set_kernel(int m, int n, const double2* __restrict__ A, int lda, const double2* __restrict__ x,
                   double2* __restrict__ y, double2 alpha, int lower) {
    __shared__ double2 part[16][17];
    const int tr = threadIdx.x & 15, cg = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + tr;
    const int jend = lower ? min(n, i + 1) : n;
    double sr = 0.0, si = 0.0;
    if (i < m) {
        const double2* a = A + i;
#pragma unroll 4
        for (int j = cg; j < jend; j += 16) {
            const double2 av = a[(long)j * lda], v = x[j];
            sr = fma(av.x, v.x, fma(-av.y, v.y, sr));
            si = fma(av.x, v.y, fma(av.y, v.x, si));
        }
    }
    part[cg][tr] = make_double2(sr, si);
    __syncthreads();
    if (cg == 0 && i < m) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) { ar += part[q][tr].x; ai += part[q][tr].y; }
        y[i] = make_double2(alpha.x * ar - alpha.y * ai, alpha.x * ai + alpha.y * ar);
    }
}

// y = beta y; beta = 0 overwrites y with zeros without reading it (y may hold
// anything, NaN included, when the caller asks for y = A x)
__global__ void zscale_kernel(int m, double2* y, double2 beta) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    if (beta.x == 0.0 && beta.y == 0.0) {
        y[i] = make_double2(0.0, 0.0);
        return;
    }
    const double2 c = y[i];
    y[i] = make_double2(beta.x * c.x - beta.y * c.y, beta.x * c.y + beta.y * c.x);
}

// out[slot] += sum |v|^2 (one workgroup per 256*16 entries, double atomics)
__global__ void __launch_bounds__(256) znorm2_kernel(int m, const double2* __restrict__ v, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
        const double2 a = v[i];
        s += a.x * a.x + a.y * a.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// normalise v (length n <= 64k) to unit norm in one workgroup, store the old norm
__global__ void __launch_bounds__(256) znormalize_kernel(int n, double2* v, double* norm_out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += v[i].x * v[i].x + v[i].y * v[i].y;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double nrm = sqrt(red[0]);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = threadIdx.x; i < n; i += 256) { v[i].x *= inv; v[i].y *= inv; }
    if (threadIdx.x == 0) *norm_out = nrm;
}

// scale columns by 1/s (s from col_norms); a zero or non-finite norm raises flag bits
__global__ void scale_cols_checked_kernel(double2* A, int m, int lda, const double* __restrict__ s, int* flags) {
    const int c = blockIdx.y;
    const double v = s[c];
    const bool ok = v > 0.0 && v < 1e300;
    if (!ok) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, v == 0.0 ? 1 : 2);
        return;
    }
    const double f = 1.0 / v;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < m; r += gridDim.x * blockDim.x) {
        double2* p = A + r + (long)c * lda;
        p->x *= f;
        p->y *= f;
    }
}

// ---------------------------------------------------------------- packed (block-sparse) interface matrix
// Qbar's rows of subdomain i only touch the unknown blocks of that subdomain,
// so it is stored as one dense block A_i (m_i x s_i, column-major) per
// subdomain.  Packed column pc (global numbering over all subdomains) belongs
// to subdomain pc_sub[pc], is column pc_p[pc] of its block and column
// pc_gcol[pc] of Qbar; it is coefA Q_i(:, colA) + coefB Q_i(:, colB).
struct PackedDesc {
    const double2* const* Q;   // per subdomain: its projector's Q (ld = m_i)
    const int* m;              // rows per subdomain
    const long* off;           // start of A_i in the packed buffer
    const int* s;              // packed columns per subdomain
    const int* pc_sub;
    const int* pc_p;
    const int* pc_gcol;
    const int4* pc_cols;       // (colA, colB, -, -), -1 = absent
    const double2* pc_coef;    // 2 per packed column
    const long* roff;          // first row of subdomain i in the stacked right-hand side
};

// packed column pc at row r: its (at most two) Q columns combined with their coefficients
__device__ inline double2 packed_value(const PackedDesc& d, const double2* __restrict__ Q, int m, int4 cm, double2 wa,
                                       double2 wb, int r) {
    double2 v = make_double2(0.0, 0.0);
    if (cm.x >= 0) {
        const double2 q = Q[r + (long)cm.x * m];
        v.x += wa.x * q.x - wa.y * q.y;
        v.y += wa.x * q.y + wa.y * q.x;
    }
    if (cm.y >= 0) {
        const double2 q = Q[r + (long)cm.y * m];
        v.x += wb.x * q.x - wb.y * q.y;
        v.y += wb.x * q.y + wb.y * q.x;
    }
    return v;
}

// the packed blocks, each column divided by the norm of its global column; a thread takes
// kAsmRows rows 256 apart, all its loads issued before the first store
constexpr int kAsmRows = 4;
__global__ void __launch_bounds__(256) assemble_packed_kernel(PackedDesc d, const double* __restrict__ norms,
                                                              double2* __restrict__ Ap) {
    const int pc = blockIdx.y;
    const int i = d.pc_sub[pc], p = d.pc_p[pc], m = d.m[i];
    const int r0 = blockIdx.x * 256 * kAsmRows + threadIdx.x;
    if (r0 >= m) return;
    const int4 cm = d.pc_cols[pc];
    const double2 wa = d.pc_coef[2 * pc], wb = d.pc_coef[2 * pc + 1];
    const double f = 1.0 / norms[d.pc_gcol[pc]];
    const double2* Q = d.Q[i];
    double2* out = Ap + d.off[i] + (long)p * m;
    double2 v[kAsmRows];
#pragma unroll
    for (int u = 0; u < kAsmRows; ++u) {
        const int r = r0 + 256 * u;
        v[u] = r < m ? packed_value(d, Q, m, cm, wa, wb, r) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kAsmRows; ++u) {
        const int r = r0 + 256 * u;
        if (r < m) out[r] = make_double2(v[u].x * f, v[u].y * f);
    }
}

// norms2[gcol] += ||packed column||^2 from the Q columns it combines (one workgroup per
// packed column; a global column has at most two packed columns, so the atomic sum does
// not depend on their order)
__global__ void __launch_bounds__(256) packed_colnorm2_kernel(PackedDesc d, double* norms2) {
    const int pc = blockIdx.x;
    const int i = d.pc_sub[pc], m = d.m[i];
    const int4 cm = d.pc_cols[pc];
    const double2 wa = d.pc_coef[2 * pc], wb = d.pc_coef[2 * pc + 1];
    const double2* Q = d.Q[i];
    __shared__ double red[256];
    double s = 0.0;
    for (int r0 = threadIdx.x; r0 < m; r0 += 256 * kAsmRows) {   // kAsmRows loads in flight
        double2 v[kAsmRows];
#pragma unroll
        for (int u = 0; u < kAsmRows; ++u) {
            const int r = r0 + 256 * u;
            v[u] = r < m ? packed_value(d, Q, m, cm, wa, wb, r) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < kAsmRows; ++u) s += v[u].x * v[u].x + v[u].y * v[u].y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&norms2[d.pc_gcol[pc]], red[0]);
}

// norms = sqrt(norms2); zero / non-finite norms raise flag bits 1 / 2
__global__ void finalize_norms_kernel(int n, const double* __restrict__ norms2, double* norms, int* flags) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double v = norms2[c];
    if (!(v < 1e300)) { atomicOr(flags, 2); norms[c] = 1.0; return; }
    if (!(v > 0.0)) { atomicOr(flags, 1); norms[c] = 1.0; return; }
    norms[c] = sqrt(v);
}

// y[gcol] += alpha * A_i(:, p)^* v_i (one workgroup per packed column)
__global__ void __launch_bounds__(256) packed_ahx_kernel(PackedDesc d, const double2* __restrict__ Ap,
                                                         const double2* __restrict__ v, double2 alpha, double* y) {
    const int pc = blockIdx.x;
    const int i = d.pc_sub[pc], p = d.pc_p[pc], m = d.m[i];
    const double2* col = Ap + d.off[i] + (long)p * m;
    const double2* vi = v + d.roff[i];
    __shared__ double rr[256], ri[256];
    double sr = 0.0, si = 0.0;
    for (int r = threadIdx.x; r < m; r += 256) {
        const double2 a = col[r], b = vi[r];
        sr += a.x * b.x + a.y * b.y;
        si += a.x * b.y - a.y * b.x;
    }
    rr[threadIdx.x] = sr;
    ri[threadIdx.x] = si;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) { rr[threadIdx.x] += rr[threadIdx.x + w]; ri[threadIdx.x] += ri[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int g = d.pc_gcol[pc];
        atomicAdd(&y[2 * g], alpha.x * rr[0] - alpha.y * ri[0]);
        atomicAdd(&y[2 * g + 1], alpha.x * ri[0] + alpha.y * rr[0]);
    }
}

// y[g] = sum over the packed columns p of global column g (gc_list[gc_start[g] ..
// gc_start[g+1]-1]) of A_i(:, p)^* v_i: one workgroup per global column, y overwritten,
// every sum in a fixed order (no atomics).
__global__ void __launch_bounds__(256) packed_ahx_set_kernel(PackedDesc d, const double2* __restrict__ Ap,
                                                             const double2* __restrict__ v,
                                                             const int* __restrict__ gc_start,
                                                             const int* __restrict__ gc_list,
                                                             double2* __restrict__ y) {
    const int g = blockIdx.x;
    __shared__ double rr[256], ri[256];
    double sr = 0.0, si = 0.0;
    for (int e = gc_start[g]; e < gc_start[g + 1]; ++e) {
        const int pc = gc_list[e];
        const int i = d.pc_sub[pc], p = d.pc_p[pc], m = d.m[i];
        const double2* col = Ap + d.off[i] + (long)p * m;
        const double2* vi = v + d.roff[i];
#pragma unroll 4
        for (int r = threadIdx.x; r < m; r += 256) {
            const double2 a = col[r], b = vi[r];
            sr = fma(a.x, b.x, fma(a.y, b.y, sr));
            si = fma(a.x, b.y, fma(-a.y, b.x, si));
        }
    }
    rr[threadIdx.x] = sr;
    ri[threadIdx.x] = si;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) { rr[threadIdx.x] += rr[threadIdx.x + w]; ri[threadIdx.x] += ri[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) y[g] = make_double2(rr[0], ri[0]);
}

// out_i = F_i + alpha A_i x(gcol of its columns) (F null: alpha A_i x) for the rows of
// subdomain i = blockIdx.y: 32 rows x 8 column groups per workgroup, the groups'
// partial sums added in a fixed order (no atomics).  norms (if set): norms[0] +=
// ||out||^2, norms[1] += ||F||^2 over the rows (accumulators zeroed by an earlier
// kernel).  clr (if set): clr[0] = clr[1] = 0, by the first workgroup (the
// accumulators of a later kernel).
__global__ void __launch_bounds__(256) packed_axpy_kernel(PackedDesc d, const double2* __restrict__ Ap,
                                                          const double2* __restrict__ x,
                                                          const int* __restrict__ pc_start, double2 alpha,
                                                          const double2* __restrict__ F, double2* __restrict__ out,
                                                          double* norms, double* clr) {
    const int i = blockIdx.y;
    if (clr && blockIdx.x == 0 && i == 0 && threadIdx.x == 0) { clr[0] = 0.0; clr[1] = 0.0; }
    const int m = d.m[i], s = d.s[i];
    if ((int)blockIdx.x * 32 >= m) return;   // the whole workgroup
    const int tr = threadIdx.x & 31, cg = threadIdx.x >> 5;
    const int row = blockIdx.x * 32 + tr;
    __shared__ double2 part[8][33];
    __shared__ double nrm[2][32];
    double sr = 0.0, si = 0.0;
    if (row < m) {
        const double2* A = Ap + d.off[i] + row;
        const int* gc = d.pc_gcol + pc_start[i];
#pragma unroll 4
        for (int c = cg; c < s; c += 8) {
            const double2 a = A[(long)c * m], v = x[gc[c]];
            sr = fma(a.x, v.x, fma(-a.y, v.y, sr));
            si = fma(a.x, v.y, fma(a.y, v.x, si));
        }
    }
    part[cg][tr] = make_double2(sr, si);
    __syncthreads();
    if (cg == 0) {
        double rn = 0.0, fn = 0.0;
        if (row < m) {
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) { ar += part[q][tr].x; ai += part[q][tr].y; }
            const long o = d.roff[i] + row;
            const double2 f = F ? F[o] : make_double2(0.0, 0.0);
            const double2 res = make_double2(f.x + alpha.x * ar - alpha.y * ai, f.y + alpha.x * ai + alpha.y * ar);
            out[o] = res;
            rn = res.x * res.x + res.y * res.y;
            fn = f.x * f.x + f.y * f.y;
        }
        nrm[0][tr] = rn;
        nrm[1][tr] = fn;
    }
    if (!norms) return;   // uniform over the workgroup
    __syncthreads();
    if (threadIdx.x < 2) {
        double a = 0.0;
        for (int q = 0; q < 32; ++q) a += nrm[threadIdx.x][q];
        atomicAdd(&norms[threadIdx.x], a);
    }
}

// x += dx; norms (if set): norms[0] += ||x||^2 of the updated x, norms[1] += ||dx||^2
// (accumulators zeroed by an earlier kernel); clr (if set): clr[0] = clr[1] = 0 by the
// first workgroup.
__global__ void __launch_bounds__(256) zaxpy_norms_kernel(int n, const double2* __restrict__ dx,
                                                          double2* __restrict__ x, double* norms, double* clr) {
    if (clr && blockIdx.x == 0 && threadIdx.x == 0) { clr[0] = 0.0; clr[1] = 0.0; }
    __shared__ double red[2][256];
    double xn = 0.0, dn = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double2 d = dx[i];
        double2 v = x[i];
        v.x += d.x;
        v.y += d.y;
        x[i] = v;
        xn += v.x * v.x + v.y * v.y;
        dn += d.x * d.x + d.y * d.y;
    }
    if (!norms) return;   // uniform over the grid
    red[0][threadIdx.x] = xn;
    red[1][threadIdx.x] = dn;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&norms[0], red[0][0]);
        atomicAdd(&norms[1], red[1][0]);
    }
}

// r_i += alpha * A_i x(gcol of its columns): thread per row, 32-column chunks, atomics
__global__ void __launch_bounds__(256) packed_ax_kernel(PackedDesc d, const double2* __restrict__ Ap,
                                                        const double2* __restrict__ x, const int* __restrict__ pc_start,
                                                        double2 alpha, double* r) {
    const int i = blockIdx.z;
    const int m = d.m[i], s = d.s[i];
    const int row = blockIdx.x * 256 + threadIdx.x;
    const int c0 = blockIdx.y * 32;
    if (row >= m || c0 >= s) return;
    const double2* A = Ap + d.off[i];
    const int pcb = pc_start[i];
    double sr = 0.0, si = 0.0;
    const int c1 = min(s, c0 + 32);
    for (int c = c0; c < c1; ++c) {
        const double2 a = A[row + (long)c * m], v = x[d.pc_gcol[pcb + c]];
        sr += a.x * v.x - a.y * v.y;
        si += a.x * v.y + a.y * v.x;
    }
    double* o = r + 2 * (d.roff[i] + row);
    atomicAdd(&o[0], alpha.x * sr - alpha.y * si);
    atomicAdd(&o[1], alpha.x * si + alpha.y * sr);
}

// G(gcol_b(p1), gcol_b(p2)) += sum over the K splits of Gi_b(p1, p2), p1 >= p2, for
// every batch entry b (blockIdx.y): the batched Gram products reduced and
// scattered into the lower triangle of G in one pass.  An entry of G receives at
// most two contributions (a column block belongs to at most two subdomains) and
// two-term sums do not depend on their order, so the atomics are deterministic.
__global__ void gram_scatter_kernel(const ZBatch* __restrict__ zb, const double2* __restrict__ P, int nsplit,
                                    const int* __restrict__ gcol_all, double2* G, int ldg) {
    const ZBatch e = zb[blockIdx.y];
    const int n = e.n;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * n) return;
    const int p1 = (int)(t % n), p2 = (int)(t / n);
    if (p1 < p2) return;
    const double2* part = P + e.poff + t;
    const long ps = (long)n * n;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < nsplit; ++k) {
        const double2 v = part[k * ps];
        sr += v.x;
        si += v.y;
    }
    // G(g1, g2) = A_p1^* A_p2 into the lower triangle: the conjugate at (g2, g1) when the global
    // order of the two columns is the reverse of the local one
    const int* gcol = gcol_all + e.gcol_off;
    const int g1 = gcol[p1], g2 = gcol[p2];
    double* o = reinterpret_cast<double*>(g1 >= g2 ? G + g1 + (long)g2 * ldg : G + g2 + (long)g1 * ldg);
    atomicAdd(&o[0], sr);
    atomicAdd(&o[1], g1 >= g2 ? si : -si);
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

// F(r) = -sum_k Q_s(rl, kcol[k]) * kval[k] over the known coefficients of subdomain s;
// four lanes per row split the sum.
__global__ void known_rhs_kernel(const double2* const* __restrict__ Qsrc, const int* __restrict__ qld, int n_sub,
                                 const int* __restrict__ row_off, const int* __restrict__ kcol,
                                 const double2* __restrict__ kval, const int* __restrict__ koff,
                                 double2* __restrict__ F) {
    const int total_rows = row_off[n_sub];
    const long gt = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int part = (int)(gt & 3);
    const long r = gt >> 2;            // the 4 lanes of a row are adjacent in one wavefront
    double sr = 0.0, si = 0.0;
    if (r < total_rows) {
        int s = 0;
        while (r >= row_off[s + 1]) ++s;
        const int rl = (int)(r - row_off[s]);
        for (int k = koff[s] + part; k < koff[s + 1]; k += 4) {
            const double2 q = Qsrc[s][rl + (long)kcol[k] * qld[s]], w = kval[k];
            sr += w.x * q.x - w.y * q.y;
            si += w.x * q.y + w.y * q.x;
        }
    }
    sr += __shfl_xor(sr, 1, 64);
    si += __shfl_xor(si, 1, 64);
    sr += __shfl_xor(sr, 2, 64);
    si += __shfl_xor(si, 2, 64);
    if (r < total_rows && part == 0) F[r] = make_double2(-sr, -si);
}

// Full coefficient vectors from the least-squares unknowns:
// c[e] = known[e] + coef[e] x[src[e]] (src[e] < 0: known value only).
__global__ void expand_coeffs_kernel(int n, const int* __restrict__ src, const double2* __restrict__ coef,
                                     const double2* __restrict__ known, const double2* __restrict__ x,
                                     double2* __restrict__ c) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double2 v = known[e];
    const int s = src[e];
    if (s >= 0) {
        const double2 w = coef[e], u = x[s];
        v.x += w.x * u.x - w.y * u.y;
        v.y += w.x * u.y + w.y * u.x;
    }
    c[e] = v;
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
                  const double2* B, int ldb, double2 beta, double2* C, int ldc, DevBuf& P, hipStream_t st, int tri) {
    if (m <= 0 || n <= 0) return;
    if (n == 1 && tri == 0) {   // matrix-vector products
        if (opB != 'N') throw Error(MDP_ERR_ARG, "gemv with a transposed vector");
        if (opA == 'C')
            hipLaunchKernelGGL(zgemv_c_kernel, dim3(m), dim3(256), 0, st, k, A, lda, B, C, alpha, beta, 0);
        else if (beta.x == 0.0 && beta.y == 0.0) {
            hipLaunchKernelGGL(zgemv_n_set_kernel, dim3((m + 15) / 16), dim3(256), 0, st, m, k, A, lda, B, C, alpha, 0);
        } else {
            if (!(beta.x == 1.0 && beta.y == 0.0))
                hipLaunchKernelGGL(zscale_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, C, beta);
            hipLaunchKernelGGL(zgemv_n_kernel, dim3((m + 255) / 256, (k + 63) / 64), dim3(256), 0, st, m, k, A, lda,
                               B, (double*)C, alpha);
        }
        MDP_HIP(hipGetLastError());
        return;
    }
    const int oa = (opA == 'C') ? 1 : 0, ob = (opB == 'C') ? 1 : 0;
    // 64x64 tiles when they fill the chip, 32x32 for small products
    const int tile = ((long)((m + 63) / 64) * ((n + 63) / 64) >= 128) ? 64 : 32;
    const int mt = (m + tile - 1) / tile, nt = (n + tile - 1) / tile;
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
    const long pstride = (long)m * n;
    double2* part = nullptr;
    if (nsplit > 1) {
        const size_t need = (size_t)pstride * nsplit * sizeof(double2);
        if (need > P.bytes) {   // never free a buffer earlier kernels may still read
            MDP_HIP(hipDeviceSynchronize());
            P.reserve(need);
        }
        part = P.as<double2>();
    }
    if (tile == 64)
        hipLaunchKernelGGL(zgemm_kernel<64>, dim3(tiles, nsplit), dim3(256), 0, st, oa, ob, m, n, k, A, lda, B, ldb,
                           C, ldc, alpha, beta, kchunk, part, pstride, mt, tri, nullptr);
    else
        hipLaunchKernelGGL(zgemm_kernel<32>, dim3(tiles, nsplit), dim3(256), 0, st, oa, ob, m, n, k, A, lda, B, ldb,
                           C, ldc, alpha, beta, kchunk, part, pstride, mt, tri, nullptr);
    MDP_HIP(hipGetLastError());
    if (nsplit > 1) {
        hipLaunchKernelGGL(zgemm_reduce_kernel, dim3((m + 255) / 256, n), dim3(256), 0, st, m, n, nsplit, part,
                           pstride, C, ldc, alpha, beta, tri, tile);
        MDP_HIP(hipGetLastError());
    }
}

void launch_chol_diag(const double2* G, int nc, const CholStepDev& sp, double shift, double2* L, double2* Z, int* info,
                      hipStream_t st) {
    if (sp.nq < 1 || sp.nq > CholStepDev::kMaxQ || sp.kb < 0 || sp.off[0] != 0 || sp.off[sp.nq] != sp.wtot ||
        sp.kb + sp.wtot > nc)
        throw Error(MDP_ERR_ARG, "bad Cholesky step");
    for (int q = 0; q < sp.nq; ++q)
        if (sp.off[q + 1] - sp.off[q] < 1 || sp.off[q + 1] - sp.off[q] > 64)
            throw Error(MDP_ERR_ARG, "Cholesky sub-block width must be 1..64");
    hipLaunchKernelGGL(chol_diag_kernel, dim3(sp.nq), dim3(256), 0, st, G, nc, sp, shift, L, Z, info);
    MDP_HIP(hipGetLastError());
}
void launch_chol_slabs(const double2* G, int nc, const CholStepDev& sp, double2* L, double2* Z, const double2* W,
                       hipStream_t st) {
    const int rest = nc - sp.kb - sp.wtot;
    const int np = (rest + 31) / 32, nz = (sp.kb + 31) / 32;
    if (np + nz == 0) return;
    hipLaunchKernelGGL(chol_slab_kernel, dim3(sp.nq * (np + nz)), dim3(256), 0, st, G, nc, sp, L, Z, W, np, nz);
    MDP_HIP(hipGetLastError());
}
void launch_chol_diag_batched(const CholBatchEntry* ent, int count, int* info, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(chol_diag_batched_kernel, dim3(count), dim3(256), 0, st, ent, info);
    MDP_HIP(hipGetLastError());
}
void launch_chol_slabs_batched(const CholBatchEntry* ent, int count, int max_roles, hipStream_t st) {
    if (count <= 0 || max_roles <= 0) return;
    hipLaunchKernelGGL(chol_slab_batched_kernel, dim3(max_roles, count), dim3(256), 0, st, ent);
    MDP_HIP(hipGetLastError());
}
// 64 x 64 tiles when they still give every CU a few workgroups, else 32 x 32
void launch_chol_update_batched(const CholBatchEntry* ent, int count, int max_tiles64, long tiles64, int max_tiles32,
                                hipStream_t st) {
    if (count <= 0 || max_tiles32 <= 0) return;
    if (tiles64 >= kUpdWideMin)
        hipLaunchKernelGGL(chol_update_batched_kernel<true>, dim3(max_tiles64, count), dim3(256), 0, st, ent);
    else
        hipLaunchKernelGGL(chol_update_batched_kernel<false>, dim3(max_tiles32, count), dim3(256), 0, st, ent);
    MDP_HIP(hipGetLastError());
}
void launch_chol_update(double2* G, int nc, int kb, int wtot, const double2* L, const double2* Z, double2* W,
                        hipStream_t st) {
    const int t64 = chol_update_tiles(nc, kb, wtot, 64), t32 = chol_update_tiles(nc, kb, wtot, 32);
    if (t32 <= 0) return;
    if (t64 >= kUpdWideMin)
        hipLaunchKernelGGL(chol_update_kernel<true>, dim3(t64), dim3(256), 0, st, G, nc, kb, wtot, L, Z, W);
    else
        hipLaunchKernelGGL(chol_update_kernel<false>, dim3(t32), dim3(256), 0, st, G, nc, kb, wtot, L, Z, W);
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
    const unsigned blocks = (unsigned)(((long)total_rows * 4 + 255) / 256);
    if (total_rows <= 0) return;
    hipLaunchKernelGGL(known_rhs_kernel, dim3(blocks), dim3(256), 0, st, Qsrc, qld, n_sub, row_off, kcol, kval, koff,
                       F);
    MDP_HIP(hipGetLastError());
}

void launch_expand_coeffs(int n, const int* src, const double2* coef, const double2* known, const double2* x,
                          double2* c, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(expand_coeffs_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, src, coef, known, x, c);
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

void launch_znorm2(int m, const double2* v, double* out, hipStream_t st) {
    int g = std::min(1024, std::max(1, (m + 4095) / 4096));
    hipLaunchKernelGGL(znorm2_kernel, dim3(g), dim3(256), 0, st, m, v, out);
    MDP_HIP(hipGetLastError());
}

void launch_znormalize(int n, double2* v, double* norm_out, hipStream_t st) {
    hipLaunchKernelGGL(znormalize_kernel, dim3(1), dim3(256), 0, st, n, v, norm_out);
    MDP_HIP(hipGetLastError());
}

void launch_scale_cols_checked(double2* A, int m, int n, int lda, const double* s, int* flags, hipStream_t st) {
    dim3 grid(std::max(1, std::min((m + 255) / 256, 64)), n);
    hipLaunchKernelGGL(scale_cols_checked_kernel, grid, dim3(256), 0, st, A, m, lda, s, flags);
    MDP_HIP(hipGetLastError());
}

void launch_assemble_packed(const PackedDevice& d, int total_pc, int max_m, const double* norms, double2* Ap,
                            hipStream_t st) {
    PackedDesc pd{d.Q, d.m, d.off, d.s, d.pc_sub, d.pc_p, d.pc_gcol, d.pc_cols, d.pc_coef, d.roff};
    dim3 grid(std::max(1, (max_m + 256 * kAsmRows - 1) / (256 * kAsmRows)), total_pc);
    hipLaunchKernelGGL(assemble_packed_kernel, grid, dim3(256), 0, st, pd, norms, Ap);
    MDP_HIP(hipGetLastError());
}

void launch_packed_colnorm2(const PackedDevice& d, int total_pc, double* norms2, hipStream_t st) {
    PackedDesc pd{d.Q, d.m, d.off, d.s, d.pc_sub, d.pc_p, d.pc_gcol, d.pc_cols, d.pc_coef, d.roff};
    hipLaunchKernelGGL(packed_colnorm2_kernel, dim3(total_pc), dim3(256), 0, st, pd, norms2);
    MDP_HIP(hipGetLastError());
}

void launch_finalize_norms(int n, const double* norms2, double* norms, int* flags, hipStream_t st) {
    hipLaunchKernelGGL(finalize_norms_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, norms2, norms, flags);
    MDP_HIP(hipGetLastError());
}

void launch_packed_ahx(const PackedDevice& d, int total_pc, const double2* Ap, const double2* v, double2 alpha,
                       double2* y, hipStream_t st) {
    PackedDesc pd{d.Q, d.m, d.off, d.s, d.pc_sub, d.pc_p, d.pc_gcol, d.pc_cols, d.pc_coef, d.roff};
    hipLaunchKernelGGL(packed_ahx_kernel, dim3(total_pc), dim3(256), 0, st, pd, Ap, v, alpha, (double*)y);
    MDP_HIP(hipGetLastError());
}

void launch_packed_ax(const PackedDevice& d, int n_sub, int max_m, int max_s, const double2* Ap, const double2* x,
                      double2 alpha, double2* r, hipStream_t st) {
    PackedDesc pd{d.Q, d.m, d.off, d.s, d.pc_sub, d.pc_p, d.pc_gcol, d.pc_cols, d.pc_coef, d.roff};
    dim3 grid((max_m + 255) / 256, (max_s + 31) / 32, n_sub);
    hipLaunchKernelGGL(packed_ax_kernel, grid, dim3(256), 0, st, pd, Ap, x, d.pc_start, alpha, (double*)r);
    MDP_HIP(hipGetLastError());
}

void launch_gram_batched(const ZBatch* zb_dev, int nb, int max_n, int max_k, int nsplit, double2* P, const int* gcol,
                         double2* G, int ldg, hipStream_t st) {
    if (nb <= 0) return;
    // 32 x 32 workgroup tiles for a batch that gives every CU a few of them (the 16x16 layout's
    // blocks, order 256 and some 3000 rows: ~9k lower tiles); 64 x 32 for smaller batches, where
    // the longer tiles measured faster (cross-point: 0.053 against 0.063 ms) and slower on the
    // 16x16 layout; square 64 x 64 tiles measured 1.7x slower there
    const int mt = (max_n + kGramTile - 1) / kGramTile;
    const long lower32 = (long)nb * nsplit * mt * (mt + 1) / 2;
    if (lower32 >= 2048) {
        hipLaunchKernelGGL((gram_kernel<32, 32>), dim3(mt * mt, nsplit, nb), dim3(256), 0, st, zb_dev, P);
    } else {
        const int tiles = ((max_n + 63) / 64) * ((max_n + 31) / 32);
        hipLaunchKernelGGL((gram_kernel<64, 32>), dim3(tiles, nsplit, nb), dim3(256), 0, st, zb_dev, P);
    }
    MDP_HIP(hipGetLastError());
    (void)max_k;
    if (!G) return;   // the partials are used as they are (multifrontal leaves)
    hipLaunchKernelGGL(gram_scatter_kernel, dim3((unsigned)(((long)max_n * max_n + 255) / 256), nb), dim3(256), 0, st,
                       zb_dev, P, nsplit, gcol, G, ldg);
    MDP_HIP(hipGetLastError());
}

void launch_trmv_lower(char op, int n, const double2* A, int lda, const double2* x, double2* y, hipStream_t st) {
    if (n <= 0) return;
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    if (op == 'C')
        hipLaunchKernelGGL(zgemv_c_kernel, dim3(n), dim3(256), 0, st, n, A, lda, x, y, one, zero, 1);
    else
        hipLaunchKernelGGL(zgemv_n_set_kernel, dim3((n + 15) / 16), dim3(256), 0, st, n, n, A, lda, x, y, one, 1);
    MDP_HIP(hipGetLastError());
}

void launch_packed_ahx_set(const PackedDevice& d, int nc, const double2* Ap, const double2* v, double2* y,
                           hipStream_t st) {
    if (nc <= 0) return;
    PackedDesc pd{d.Q, d.m, d.off, d.s, d.pc_sub, d.pc_p, d.pc_gcol, d.pc_cols, d.pc_coef, d.roff};
    hipLaunchKernelGGL(packed_ahx_set_kernel, dim3(nc), dim3(256), 0, st, pd, Ap, v, d.gc_start, d.gc_list, y);
    MDP_HIP(hipGetLastError());
}

void launch_packed_axpy(const PackedDevice& d, int n_sub, int max_m, const double2* Ap, const double2* x,
                        double2 alpha, const double2* F, double2* out, double* norms, double* clr, hipStream_t st) {
    if (n_sub <= 0 || max_m <= 0) return;
    PackedDesc pd{d.Q, d.m, d.off, d.s, d.pc_sub, d.pc_p, d.pc_gcol, d.pc_cols, d.pc_coef, d.roff};
    hipLaunchKernelGGL(packed_axpy_kernel, dim3((max_m + 31) / 32, n_sub), dim3(256), 0, st, pd, Ap, x, d.pc_start,
                       alpha, F, out, norms, clr);
    MDP_HIP(hipGetLastError());
}

void launch_zaxpy_norms(int n, const double2* dx, double2* x, double* norms, double* clr, hipStream_t st) {
    const int g = std::max(1, std::min(256, (n + 255) / 256));
    hipLaunchKernelGGL(zaxpy_norms_kernel, dim3(g), dim3(256), 0, st, n, dx, x, norms, clr);
    MDP_HIP(hipGetLastError());
}

// One refinement pass over the packed matrix: the residual r = F - A_i x of the 32 rows of slab
// blockIdx.x of subdomain i = blockIdx.y (as packed_axpy_kernel with alpha = -1; r stays in LDS),
// then the slab's share of A_i^* r for every packed column c of the subdomain,
// P[(pc_start[i] + c) * ms + slab] (the slab's rows were just read: the second read hits the
// caches).  clr as in packed_axpy_kernel.
__global__ void __launch_bounds__(256) packed_resid_ahx_kernel(PackedDesc d, const double2* __restrict__ Ap,
                                                               const double2* __restrict__ x,
                                                               const int* __restrict__ pc_start,
                                                               const double2* __restrict__ F,
                                                               double2* __restrict__ P, int ms, double* clr) {
    const int i = blockIdx.y;
    if (clr && blockIdx.x == 0 && i == 0 && threadIdx.x == 0) { clr[0] = 0.0; clr[1] = 0.0; }
    const int m = d.m[i], s = d.s[i];
    const int row0 = blockIdx.x * 32;
    if (row0 >= m) return;   // the whole workgroup
    const int tr = threadIdx.x & 31, cg = threadIdx.x >> 5;
    const int row = row0 + tr;
    __shared__ double2 part[8][33];
    __shared__ double2 rs[32];
    const double2* __restrict__ Ai = Ap + d.off[i];
    double sr = 0.0, si = 0.0;
    if (row < m) {
        const double2* A = Ai + row;
        const int* gc = d.pc_gcol + pc_start[i];
#pragma unroll 4
        for (int c = cg; c < s; c += 8) {
            const double2 a = A[(long)c * m], v = x[gc[c]];
            sr = fma(a.x, v.x, fma(-a.y, v.y, sr));
            si = fma(a.x, v.y, fma(a.y, v.x, si));
        }
    }
    part[cg][tr] = make_double2(sr, si);
    __syncthreads();
    if (cg == 0) {
        double2 res = make_double2(0.0, 0.0);
        if (row < m) {
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) { ar += part[q][tr].x; ai += part[q][tr].y; }
            const double2 f = F[d.roff[i] + row];
            res = make_double2(f.x - ar, f.y - ai);
        }
        rs[tr] = res;
    }
    __syncthreads();
    const int nr = min(32, m - row0);
    double2* __restrict__ Pi = P + (long)pc_start[i] * ms + blockIdx.x;
    for (int c = threadIdx.x; c < s; c += 256) {
        const double2* col = Ai + (long)c * m + row0;
        double pr = 0.0, pi = 0.0;
        if (nr == 32) {
#pragma unroll 8
            for (int k = 0; k < 32; ++k) {
                const double2 a = col[k], b = rs[k];
                pr = fma(a.x, b.x, fma(a.y, b.y, pr));
                pi = fma(a.x, b.y, fma(-a.y, b.x, pi));
            }
        } else {
            for (int k = 0; k < nr; ++k) {
                const double2 a = col[k], b = rs[k];
                pr = fma(a.x, b.x, fma(a.y, b.y, pr));
                pi = fma(a.x, b.y, fma(-a.y, b.x, pi));
            }
        }
        Pi[(long)c * ms] = make_double2(pr, pi);
    }
}

// The same pass for subdomains of at most 256 packed columns, every entry of the slab read once:
// thread t holds rows (t & 7) + 8 q (q < 4) of columns 8 (t >> 3) .. +7 of the 32 x 256 slab in
// registers (eight consecutive lanes read 128 consecutive bytes of a column); the row sums (over the 32 column groups) and, once r is known, the
// column sums (over the 8 row groups) are added in LDS in a fixed order.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) packed_resid_ahx_reg_kernel(PackedDesc d, const double2* __restrict__ Ap,
                                                                   const double2* __restrict__ x,
                                                                   const int* __restrict__ pc_start,
                                                                   const double2* __restrict__ F,
                                                                   double2* __restrict__ P, int ms, double* clr) {
    const int i = blockIdx.y;
    if (clr && blockIdx.x == 0 && i == 0 && threadIdx.x == 0) { clr[0] = 0.0; clr[1] = 0.0; }
    const int m = d.m[i], s = d.s[i];
    const int row0 = blockIdx.x * 32;
    if (row0 >= m) return;   // the whole workgroup
    const int t = threadIdx.x, rg = t & 7, cq = t >> 3;
    __shared__ double2 red1[32][33];   // [column group][row]
    __shared__ double2 red2[8][257];   // [row group][column]
    __shared__ double2 rs[32];
    const double2* __restrict__ Ai = Ap + d.off[i];
    const int* __restrict__ gc = d.pc_gcol + pc_start[i];
    double2 a[8][4], xv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int c = 8 * cq + j;
        const bool cin = c < s;
        xv[j] = cin ? x[gc[c]] : make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = row0 + rg + 8 * q;
            a[j][q] = (cin && row < m) ? Ai[row + (long)c * m] : make_double2(0.0, 0.0);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {   // the block's share of (A x)(row)
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sr = fma(a[j][q].x, xv[j].x, fma(-a[j][q].y, xv[j].y, sr));
            si = fma(a[j][q].x, xv[j].y, fma(a[j][q].y, xv[j].x, si));
        }
        red1[cq][rg + 8 * q] = make_double2(sr, si);
    }
    __syncthreads();
    if (t < 32) {
        double2 res = make_double2(0.0, 0.0);
        if (row0 + t < m) {
            double ar = 0.0, ai = 0.0;
            for (int g = 0; g < 32; ++g) { ar += red1[g][t].x; ai += red1[g][t].y; }
            const double2 f = F[d.roff[i] + row0 + t];
            res = make_double2(f.x - ar, f.y - ai);
        }
        rs[t] = res;
    }
    __syncthreads();
    double2 rv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rv[q] = rs[rg + 8 * q];
#pragma unroll
    for (int j = 0; j < 8; ++j) {   // the block's share of (A^* r)(column)
        double pr = 0.0, pi = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pr = fma(a[j][q].x, rv[q].x, fma(a[j][q].y, rv[q].y, pr));
            pi = fma(a[j][q].x, rv[q].y, fma(-a[j][q].y, rv[q].x, pi));
        }
        red2[rg][8 * cq + j] = make_double2(pr, pi);
    }
    __syncthreads();
    if (t < s) {
        double pr = 0.0, pi = 0.0;
#pragma unroll
        for (int g = 0; g < 8; ++g) { pr += red2[g][t].x; pi += red2[g][t].y; }
        P[((long)pc_start[i] + t) * ms + blockIdx.x] = make_double2(pr, pi);
    }
}

// y[g] = sum over the packed columns pc of global column g (gc_list[gc_start[g] ..
// gc_start[g+1]-1]) and over the slabs of their subdomain of the partials P[pc * ms + slab]:
// one wavefront per global column, lanes over the slabs, a fixed summation order; y overwritten.
__global__ void __launch_bounds__(256) packed_ahx_partials_kernel(PackedDesc d, const double2* __restrict__ P, int ms,
                                                                  const int* __restrict__ gc_start,
                                                                  const int* __restrict__ gc_list, int nc,
                                                                  double2* __restrict__ y) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (g >= nc) return;   // the whole wavefront
    double sr = 0.0, si = 0.0;
    for (int e = gc_start[g]; e < gc_start[g + 1]; ++e) {
        const int pc = gc_list[e];
        const int ns = (d.m[d.pc_sub[pc]] + 31) / 32;
        for (int q = lane; q < ns; q += 64) {
            const double2 v = P[(long)pc * ms + q];
            sr += v.x;
            si += v.y;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o);
        si += __shfl_xor(si, o);
    }
    if (lane == 0) y[g] = make_double2(sr, si);
}

// out = a - b (complex vectors of length n; out may alias either)
__global__ void __launch_bounds__(256) zsub_kernel(int n, const double2* a, const double2* b, double2* out) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double2 x = a[i], y = b[i];
        out[i] = make_double2(x.x - y.x, x.y - y.y);
    }
}

void launch_packed_resid_ahx(const PackedDevice& d, int n_sub, int max_m, int max_s, int nc, const double2* Ap,
                             const double2* x, const double2* F, double2* P, double2* y, double* clr,
                             hipStream_t st) {
    if (n_sub <= 0 || max_m <= 0 || nc <= 0) return;
    PackedDesc pd{d.Q, d.m, d.off, d.s, d.pc_sub, d.pc_p, d.pc_gcol, d.pc_cols, d.pc_coef, d.roff};
    const int ms = packed_slabs(max_m);
    if (max_s <= 256)
        hipLaunchKernelGGL(packed_resid_ahx_reg_kernel, dim3(ms, n_sub), dim3(256), 0, st, pd, Ap, x, d.pc_start, F,
                           P, ms, clr);
    else
        hipLaunchKernelGGL(packed_resid_ahx_kernel, dim3(ms, n_sub), dim3(256), 0, st, pd, Ap, x, d.pc_start, F, P,
                           ms, clr);
    MDP_HIP(hipGetLastError());
    hipLaunchKernelGGL(packed_ahx_partials_kernel, dim3((nc + 3) / 4), dim3(256), 0, st, pd, P, ms, d.gc_start,
                       d.gc_list, nc, y);
    MDP_HIP(hipGetLastError());
}

void launch_zsub(int n, const double2* a, const double2* b, double2* out, hipStream_t st) {
    if (n <= 0) return;
    const int g = std::max(1, std::min(256, (n + 255) / 256));
    hipLaunchKernelGGL(zsub_kernel, dim3(g), dim3(256), 0, st, n, a, b, out);
    MDP_HIP(hipGetLastError());
}

void launch_diag_range(const double2* L, int n, int ld, double* out, hipStream_t st) {
    hipLaunchKernelGGL(diag_range_kernel, dim3(1), dim3(256), 0, st, L, n, ld, out);
    MDP_HIP(hipGetLastError());
}

void launch_fill(double* p, long n, double v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n)), dim3(256), 0, st, p, n, v);
    MDP_HIP(hipGetLastError());
}


// ---------------------------------------------------------------------------
// Multifrontal Cholesky of the interface Gram matrix (elimination tree over
// the subdomains).  Fronts are assembled by gathering: each entry of a node's
// front is the sum of at most two children's contribution entries (or one entry
// of a leaf's Gram block), so no two threads write one entry.

__global__ void __launch_bounds__(256)
mf_assemble_kernel(const MFNodeDev* __restrict__ nodes, const int* __restrict__ list, const char* __restrict__ img,
                   const double2* __restrict__ P, double2* __restrict__ arena) {
    const MFNodeDev nd = nodes[list[blockIdx.y]];
    const int f = nd.f;
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)f * f) return;
    const int a = (int)(t % f), c = (int)(t / f);   // row a, column c
    double2 v = make_double2(0.0, 0.0);
    if (nd.leaf) {
        const int* sp = reinterpret_cast<const int*>(img + nd.spos);
        int p1 = sp[a], p2 = sp[c];
        const bool cj = p1 < p2;   // the partials hold the lower triangle (p1 >= p2)
        if (cj) { const int q = p1; p1 = p2; p2 = q; }
        const double2* q = P + nd.poff + p1 + (long)p2 * nd.n;
        for (int k = 0; k < nd.nsplit; ++k) {
            const double2 w = q[k * nd.pstride];
            v.x += w.x;
            v.y += w.y;
        }
        if (cj) v.y = -v.y;
    } else {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int* inv = reinterpret_cast<const int*>(img + (kk ? nd.inv1 : nd.inv0));
            const int ia = inv[a], ic = inv[c];
            if (ia < 0 || ic < 0) continue;
            // the child's contribution block is the lower triangle of its factored front's G(e:, e:)
            const MFNodeDev& kd = nodes[kk ? nd.kid1 : nd.kid0];
            const bool lo = ia >= ic;
            const int r = kd.e + (lo ? ia : ic), cc = kd.e + (lo ? ic : ia);
            const double2 w = arena[kd.G + r + (long)cc * kd.f];
            v.x += w.x;
            v.y += lo ? w.y : -w.y;
        }
    }
    arena[nd.G + a + (long)c * f] = v;
}

__device__ inline double2 wave_sum2(double2 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    return v;
}

// Substitutions with many workgroups per node (a node's rows or columns cut into
// chunks), two launches per direction and height.  w(a), the front's right-hand
// side at position a, is y at the eliminated columns plus the children's
// contributions, gathered per position through the inverse maps.
__device__ inline double2 mf_front_rhs(const MFNodeDev& nd, const MFNodeDev* __restrict__ nodes,
                                       const char* __restrict__ img, const double2* __restrict__ arena,
                                       const double2* __restrict__ y, const int* __restrict__ idx, int a) {
    double2 v = (a < nd.e) ? y[idx[a]] : make_double2(0.0, 0.0);
    if (!nd.leaf) {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int r = reinterpret_cast<const int*>(img + (kk ? nd.inv1 : nd.inv0))[a];
            if (r < 0) continue;
            const double2 u = arena[nodes[kk ? nd.kid1 : nd.kid0].cw + r];
            v.x += u.x;
            v.y += u.y;
        }
    }
    return v;
}

// The four substitution products are bandwidth-bound matrix-vector products with
// the node's stored blocks (column-major, leading dimension f): many small
// workgroups, each with several loads in flight per thread, so that every
// height's launch spreads over the chip.
constexpr int kMfRows = 8;                   // rows of z or cw per workgroup
constexpr int kMfSlots = 256 / kMfRows;      // column slots of a row (threads per row)
constexpr int kMfCols = 4;                   // columns of t or x per workgroup (a wavefront each)

// acc += l * u (complex), or conj(l) * u
__device__ inline void cmac(double& sr, double& si, double2 l, double2 u) {
    sr = fma(l.x, u.x, fma(-l.y, u.y, sr));
    si = fma(l.x, u.y, fma(l.y, u.x, si));
}
__device__ inline void cmac_conj(double& sr, double& si, double2 l, double2 u) {
    sr = fma(l.x, u.x, fma(l.y, u.y, sr));
    si = fma(l.x, u.y, fma(-l.y, u.x, si));
}

// sum_j M(i, j) v(j) over the columns j = slot, slot + kMfSlots, ... < jend of row i
// (M(i, j) = Mi[j * ld], v in LDS), eight loads in flight
__device__ inline double2 mf_row_dot(const double2* __restrict__ Mi, long ld, const double2* v, int slot, int jend) {
    double sr = 0.0, si = 0.0;
    int j = slot;
    for (; j + 7 * kMfSlots < jend; j += 8 * kMfSlots) {
        double2 l[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) l[q] = Mi[(long)(j + q * kMfSlots) * ld];
#pragma unroll
        for (int q = 0; q < 8; ++q) cmac(sr, si, l[q], v[j + q * kMfSlots]);
    }
    for (; j < jend; j += kMfSlots) cmac(sr, si, Mi[(long)j * ld], v[j]);
    return make_double2(sr, si);
}

// the kMfSlots partial sums of each of the workgroup's kMfRows rows, added in LDS; the
// total of row r is returned to thread r (other threads: zero)
__device__ inline double2 mf_rows_total(double2 p, int r, int slot) {
    __shared__ double2 part[kMfSlots][kMfRows];
    part[slot][r] = p;
    __syncthreads();
    double2 t = make_double2(0.0, 0.0);
    if (threadIdx.x < kMfRows) {
        for (int q = 0; q < kMfSlots; ++q) {
            t.x += part[q][threadIdx.x].x;
            t.y += part[q][threadIdx.x].y;
        }
    }
    return t;
}

// z(i) = sum_{j <= i} Linv(i, j) w(j) for the kMfRows rows of chunk blockIdx.x: thread (row
// tid % kMfRows, slot tid / kMfRows) takes every kMfSlots-th column
__global__ void __launch_bounds__(256)
mf_fwd_z_kernel(const MFNodeDev* __restrict__ nodes, const int* __restrict__ list, const char* __restrict__ img,
                double2* __restrict__ arena, const double2* __restrict__ y) {
    extern __shared__ double2 mf_sh[];
    const MFNodeDev nd = nodes[list[blockIdx.y]];
    const int e = nd.e, i0 = blockIdx.x * kMfRows;
    if (i0 >= e) return;
    const int iend = min(e, i0 + kMfRows), tid = threadIdx.x, r = tid % kMfRows, slot = tid / kMfRows;
    const int* idx = reinterpret_cast<const int*>(img + nd.idx);
    for (int a = tid; a < iend; a += 256) mf_sh[a] = mf_front_rhs(nd, nodes, img, arena, y, idx, a);
    __syncthreads();
    const int i = i0 + r;
    const double2 p = (i < iend) ? mf_row_dot(arena + nd.Z + i, nd.f, mf_sh, slot, i + 1) : make_double2(0.0, 0.0);
    const double2 zz = mf_rows_total(p, r, slot);
    if (tid < kMfRows && i0 + tid < iend) arena[nd.z + i0 + tid] = zz;
}

// cw(r) = w(e + r) - sum_j L21(r, j) z(j) for the kMfRows rows of chunk blockIdx.x
__global__ void __launch_bounds__(256)
mf_fwd_cw_kernel(const MFNodeDev* __restrict__ nodes, const int* __restrict__ list, const char* __restrict__ img,
                 double2* __restrict__ arena, const double2* __restrict__ y) {
    extern __shared__ double2 mf_sh[];
    const MFNodeDev nd = nodes[list[blockIdx.y]];
    const int e = nd.e, b = nd.b, r0 = blockIdx.x * kMfRows;
    if (r0 >= b) return;
    const int tid = threadIdx.x, r = tid % kMfRows, slot = tid / kMfRows;
    const int* idx = reinterpret_cast<const int*>(img + nd.idx);
    for (int j = tid; j < e; j += 256) mf_sh[j] = arena[nd.z + j];
    __syncthreads();
    const double2 p = (r0 + r < b) ? mf_row_dot(arena + nd.L + e + r0 + r, nd.f, mf_sh, slot, e) : make_double2(0.0, 0.0);
    const double2 s = mf_rows_total(p, r, slot);
    if (tid < kMfRows && r0 + tid < b) {
        const double2 v = mf_front_rhs(nd, nodes, img, arena, y, idx, e + r0 + tid);
        arena[nd.cw + r0 + tid] = make_double2(v.x - s.x, v.y - s.y);
    }
}

// t(j) = z(j) - sum_r conj(L21(r, j)) x(idx(e + r)) for the kMfCols columns of chunk blockIdx.x (a
// wavefront per column, lanes along the column); t overwrites z
__global__ void __launch_bounds__(256)
mf_bwd_t_kernel(const MFNodeDev* __restrict__ nodes, const int* __restrict__ list, const char* __restrict__ img,
                double2* __restrict__ arena, const double2* __restrict__ x) {
    extern __shared__ double2 mf_sh[];
    const MFNodeDev nd = nodes[list[blockIdx.y]];
    const int e = nd.e, b = nd.b, f = nd.f, c0 = blockIdx.x * kMfCols;
    if (c0 >= e) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int* idx = reinterpret_cast<const int*>(img + nd.idx);
    for (int r = tid; r < b; r += 256) mf_sh[r] = x[idx[e + r]];
    __syncthreads();
    const int j = c0 + wave;
    if (j >= e) return;
    const double2* col = arena + nd.L + e + (long)j * f;
    double sr = 0.0, si = 0.0;
    int r = lane;
    for (; r + 192 < b; r += 256) {
        double2 l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) l[q] = col[r + 64 * q];
#pragma unroll
        for (int q = 0; q < 4; ++q) cmac_conj(sr, si, l[q], mf_sh[r + 64 * q]);
    }
    for (; r < b; r += 64) cmac_conj(sr, si, col[r], mf_sh[r]);
    const double2 s = wave_sum2(make_double2(sr, si));
    if (lane == 0) {
        const double2 z = arena[nd.z + j];
        arena[nd.z + j] = make_double2(z.x - s.x, z.y - s.y);
    }
}

// x(idx(i)) = sum_{j >= i} conj(Linv(j, i)) t(j) for the kMfCols rows of chunk blockIdx.x
__global__ void __launch_bounds__(256)
mf_bwd_x_kernel(const MFNodeDev* __restrict__ nodes, const int* __restrict__ list, const char* __restrict__ img,
                const double2* __restrict__ arena, double2* __restrict__ x) {
    extern __shared__ double2 mf_sh[];
    const MFNodeDev nd = nodes[list[blockIdx.y]];
    const int e = nd.e, f = nd.f, c0 = blockIdx.x * kMfCols;
    if (c0 >= e) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int* idx = reinterpret_cast<const int*>(img + nd.idx);
    for (int j = c0 + tid; j < e; j += 256) mf_sh[j - c0] = arena[nd.z + j];
    __syncthreads();
    const int i = c0 + wave;
    if (i >= e) return;
    const double2* col = arena + nd.Z + (long)i * f;
    double sr = 0.0, si = 0.0;
    int j = i + lane;
    for (; j + 192 < e; j += 256) {
        double2 l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) l[q] = col[j + 64 * q];
#pragma unroll
        for (int q = 0; q < 4; ++q) cmac_conj(sr, si, l[q], mf_sh[j + 64 * q - c0]);
    }
    for (; j < e; j += 64) cmac_conj(sr, si, col[j], mf_sh[j - c0]);
    const double2 s = wave_sum2(make_double2(sr, si));
    if (lane == 0) x[idx[i]] = s;
}

void launch_mf_solve(const MFNodeDev* nodes, const int* list, int count, int max_e, int max_b, bool forward,
                     const char* img, double2* arena, const double2* in, double2* out, hipStream_t st) {
    if (count <= 0) return;
    const size_t lds_e = (size_t)std::max(max_e, 1) * sizeof(double2), lds_b = (size_t)std::max(max_b, 1) * sizeof(double2);
    if (forward) {
        if (max_e > 0)
            hipLaunchKernelGGL(mf_fwd_z_kernel, dim3((max_e + kMfRows - 1) / kMfRows, count), dim3(256), lds_e, st,
                               nodes, list, img, arena, in);
        if (max_b > 0)
            hipLaunchKernelGGL(mf_fwd_cw_kernel, dim3((max_b + kMfRows - 1) / kMfRows, count), dim3(256), lds_e, st,
                               nodes, list, img, arena, in);
    } else if (max_e > 0) {
        hipLaunchKernelGGL(mf_bwd_t_kernel, dim3((max_e + kMfCols - 1) / kMfCols, count), dim3(256), lds_b, st,
                           nodes, list, img, arena, (const double2*)out);
        hipLaunchKernelGGL(mf_bwd_x_kernel, dim3((max_e + kMfCols - 1) / kMfCols, count), dim3(256), lds_e, st,
                           nodes, list, img, (const double2*)arena, out);
    }
    MDP_HIP(hipGetLastError());
}

void launch_mf_assemble(const MFNodeDev* nodes, const int* list, int count, int max_f, const char* img,
                        const double2* P, double2* arena, hipStream_t st) {
    if (count <= 0 || max_f <= 0) return;
    const unsigned bx = (unsigned)(((long)max_f * max_f + 255) / 256);
    hipLaunchKernelGGL(mf_assemble_kernel, dim3(bx, count), dim3(256), 0, st, nodes, list, img, P, arena);
    MDP_HIP(hipGetLastError());
}

}  // namespace mdp
