// Block-diagonal GEMM on MFMA for the folded type-I sine transform.
//
// C[M x W] = A[M x W] * B[W x W] where B = diag(S1, S2) holds the sine
// sub-matrices of the odd and even modes (the two column blocks of the folded
// layout, widths P1 and P2 = W - P1).  Every row of A is one grid row of one
// right-hand side (all rows m = 0..n of all batched solves), so M = rows x
// batch is large and the contraction length is ~n/2: a dense contraction over
// many right-hand sides, the part of the auxiliary-problem solve that belongs
// on the matrix cores (paper Sec. 3.2.1: sine transform in y).
//
// Tiling (gfx950, wave64): 256 threads = 4 waves, workgroup tile BM x BN,
// each wave a (BM/WGM) x (BN/WGN) sub-tile of 16x16 MFMA blocks
// (v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32, K = 4 per instruction).
// A and B tiles are staged through LDS (double-buffered, k-major so that an
// MFMA operand fetch reads 16 consecutive elements per k row).  The N tile
// decides the K range (block-diagonal B), so no flops are spent on the zero
// off-diagonal blocks.  Workgroup ids are remapped so that the N tiles of one
// M tile run on the same XCD and share the A rows in that XCD's L2.
#include <type_traits>

#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

#include "mdp_internal.h"

namespace mdp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

template <class T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4 acc;
    typedef d2v vec;       // 16-byte global load
    static constexpr int VW = 2;
    __device__ static inline acc op(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // D layout: lane holds column (lane & 15), rows (lane >> 4) + 4 r
    __device__ static inline int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
    typedef f4 acc;
    typedef f4 vec;
    static constexpr int VW = 4;
    __device__ static inline acc op(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // D layout: lane holds column (lane & 15), rows 4 (lane >> 4) + r
    __device__ static inline int row(int lk, int r) { return 4 * lk + r; }
};

template <int Q> __device__ inline double comp(const d2v& v) { return v[Q]; }
template <int Q> __device__ inline float comp(const f4& v) { return v[Q]; }

// compile-time loop: f(integral_constant<int, I>) for I = 0..N-1
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

__device__ inline int xcd_remap(int bid, int total) {
    // consecutive workgroups are dispatched round-robin over the 8 XCDs;
    // give each XCD a contiguous range of tile ids
    const int NX = 8;
    const int per = total / NX;
    if (bid >= per * NX) return bid;
    return (bid % NX) * per + bid / NX;
}

template <class T, int BM, int BN, int BK, int WGM, int WGN>
__global__ void __launch_bounds__(256)
gemm_bd_kernel(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C, long M, int W, int P1,
               int mtiles, int ntiles) {
    using MF = Mfma<T>;
    using acc_t = typename MF::acc;
    using vec_t = typename MF::vec;
    constexpr int VW = MF::VW;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int PAD = 4;
    constexpr int VPR_A = BK / VW;                 // vectors per A-tile row
    constexpr int NA = BM * VPR_A / 256;           // A vectors per thread
    constexpr int VPR_B = BN / VW;                 // vectors per B-tile row
    constexpr int NB = BK * VPR_B / 256;           // B vectors per thread
    static_assert(NA >= 1 && NB >= 1, "tile too small for 256 threads");

    __shared__ T As[2][BK][BM + PAD];
    __shared__ T Bs[2][BK][BN + PAD];

    const int total = mtiles * ntiles;
    const int tile = xcd_remap(blockIdx.x, total);
    const int mt = tile / ntiles, nt = tile % ntiles;
    const long m0 = (long)mt * BM;
    const int n0 = nt * BN;
    const int kbeg = (n0 < P1) ? 0 : P1;
    const int kend = (n0 < P1) ? P1 : W;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave / WGN, wn = wave % WGN;
    const int lr = lane & 15, lk = lane >> 4;

    acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    vec_t ra[NA], rb[NB];

    auto gload = [&](int k0) __attribute__((always_inline)) {
        static_for<0, NA>([&](auto vv) {
            constexpr int v = decltype(vv)::value;
            int idx = tid + v * 256;
            int row = idx / VPR_A, kv = idx % VPR_A;
            long gr = m0 + row;
            ra[v] = (gr < M) ? *reinterpret_cast<const vec_t*>(A + gr * W + k0 + kv * VW) : vec_t{};
        });
        static_for<0, NB>([&](auto vv) {
            constexpr int v = decltype(vv)::value;
            int idx = tid + v * 256;
            int kr = idx / VPR_B, nv = idx % VPR_B;
            rb[v] = *reinterpret_cast<const vec_t*>(B + (long)(k0 + kr) * W + n0 + nv * VW);
        });
    };
    auto lstore = [&](int b) __attribute__((always_inline)) {
        static_for<0, NA>([&](auto vv) {
            constexpr int v = decltype(vv)::value;
            int idx = tid + v * 256;
            int row = idx / VPR_A, kv = idx % VPR_A;
            As[b][kv * VW + 0][row] = comp<0>(ra[v]);
            As[b][kv * VW + 1][row] = comp<1>(ra[v]);
            if constexpr (VW == 4) {
                As[b][kv * VW + 2][row] = comp<2>(ra[v]);
                As[b][kv * VW + 3][row] = comp<3>(ra[v]);
            }
        });
        static_for<0, NB>([&](auto vv) {
            constexpr int v = decltype(vv)::value;
            int idx = tid + v * 256;
            int kr = idx / VPR_B, nv = idx % VPR_B;
            *reinterpret_cast<vec_t*>(&Bs[b][kr][nv * VW]) = rb[v];
        });
    };

    gload(kbeg);
    lstore(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        const bool more = (k0 + BK) < kend;
        if (more) gload(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            T a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[buf][kk * 4 + lk][wm * WM + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[buf][kk * 4 + lk][wn * WN + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = MF::op(a[i], b[j], acc[i][j]);
        }
        if (more) lstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    // D layout of the 16x16 MFMA block (differs between the f64 and f32 instructions)
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            long gr = m0 + wm * WM + i * 16 + MF::row(lk, r);
            if (gr >= M) continue;
            T* crow = C + gr * W + n0 + wn * WN + lr;
#pragma unroll
            for (int j = 0; j < TN; ++j) crow[j * 16] = acc[i][j][r];
        }
    }
}

template <class T, int BM, int BN, int WGM, int WGN>
void launch_cfg(const T* A, const T* B, T* C, long M, const Fold& f, hipStream_t st) {
    constexpr int BK = 16;
    if (f.P1 % BN || f.P2 % BN || f.P1 % BK || f.P2 % BK) throw Error(MDP_ERR_ARG, "fold widths not tileable");
    const long mt = (M + BM - 1) / BM;
    const int nt = f.W / BN;
    if (mt * nt > 0x7fffffffL) throw Error(MDP_ERR_ARG, "GEMM grid too large");
    hipLaunchKernelGGL((gemm_bd_kernel<T, BM, BN, BK, WGM, WGN>), dim3((unsigned)(mt * nt)), dim3(256), 0, st, A, B,
                       C, M, f.W, f.P1, (int)mt, nt);
    MDP_HIP(hipGetLastError());
}

// Tile shapes: 0 = 128 x 128, 1 = 128 x 64, 2 = 64 x 64.
template <class T>
void launch_shape(int shape, const T* A, const T* B, T* C, long M, const Fold& f, hipStream_t st) {
    if (shape == 0) launch_cfg<T, 128, 128, 2, 2>(A, B, C, M, f, st);
    else if (shape == 1) launch_cfg<T, 128, 64, 4, 1>(A, B, C, M, f, st);
    else launch_cfg<T, 64, 64, 2, 2>(A, B, C, M, f, st);
}

// Autotuner: the tile shape of every (precision, n, rows within a factor of two), picked at
// first use by timing each eligible shape on the call's own operands (3 launches each after
// one warm-up, HIP events on the call's stream; the chosen shape runs last, so C holds its
// product).  The shapes block the same sums differently: results agree to rounding.
std::atomic<int> g_autotune{0};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tuned;

template <class T>
int tuned_shape(const T* A, const T* B, T* C, long M, const Fold& f, hipStream_t st, int fallback) {
    const bool wide = f.P1 % 128 == 0 && f.P2 % 128 == 0;
    if (!wide) return 2;
    int lg = 0;
    while ((2L << lg) <= M) ++lg;
    const auto key = std::make_tuple((int)sizeof(T), f.n, lg);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) return it->second;
    }
    hipEvent_t e0, e1;
    MDP_HIP(hipEventCreate(&e0));
    MDP_HIP(hipEventCreate(&e1));
    int best = fallback;
    float best_ms = 1e30f;
    for (int shape = 0; shape < 3; ++shape) {
        launch_shape<T>(shape, A, B, C, M, f, st);
        MDP_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r) launch_shape<T>(shape, A, B, C, M, f, st);
        MDP_HIP(hipEventRecord(e1, st));
        MDP_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        MDP_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) { best_ms = ms; best = shape; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[key] = best;
    return best;
}

}  // namespace

void set_gemm_autotune(int on) { g_autotune.store(on ? 1 : 0); }

template <class T>
void launch_gemm_bd(const T* A, const T* B, T* C, long M, const Fold& f, hipStream_t st, bool may_tune) {
    if (M <= 0) return;
    // 128 x 128 tiles when they give enough workgroups to fill the chip (256 CUs), 64 x 64 otherwise
    // (short batches: a few thousand rows)
    const long big = ((M + 127) / 128) * (f.W / 128);
    const bool wide = f.P1 % 128 == 0 && f.P2 % 128 == 0;
    const int shape = (wide && big >= 512) ? 0 : (wide && big >= 256) ? 1 : 2;
    launch_shape<T>(may_tune && g_autotune.load() ? tuned_shape<T>(A, B, C, M, f, st, shape) : shape, A, B, C, M, f,
                    st);
}

template void launch_gemm_bd<double>(const double*, const double*, double*, long, const Fold&, hipStream_t, bool);
template void launch_gemm_bd<float>(const float*, const float*, float*, long, const Fold&, hipStream_t, bool);

}  // namespace mdp
