// Projector build, support-in / gamma-out form: the fused tridiagonal sweep.
//
// For projector column b (basis function j of eq. Q_construction) the right-hand
// side g = L^(h) w |_{M+} is real and lives on the two outer rings of the M+ box
// [m_lo, m_hi] x [q_lo, q_hi]; with the box symmetric in y (q_hi = n - q_lo) its
// folded sine transform (Sec. 3.2.1) on a grid row m is
//   ghat_m(c) = gA_m S(q_lo - 1, c) + gB_m S(q_lo, c)        (ring rows)
//             = spec_hat_m(c)                                 (the four dense rows
//                                                              m_lo, m_lo+1, m_hi-1, m_hi,
//                                                              transformed by the MFMA GEMM)
// with (gA, gB) the folded ring pair of the column's parity block.  Per folded
// mode column c the AP reduces to one complex tridiagonal system in x (eq.
// discrete_AP diagonalised by the sine transform), solved over the rows
// m0 = m_lo - 1 .. t = m_hi + 1 only: above the box the right-hand side and so
// the forward-eliminated y vanish, below it the rows are eliminated in advance
// (twisted pivot tw_t).  With the LU factors l_m, r_m = 1/d'_m and the real
// off-diagonal a of interior rows:
//   y_m = ghat_m - l_m y_{m-1},   x_t = tw_t y_t,   x_m = r_m (y_m - a x_{m+1}).
// Q needs the solution on gamma only (eq. def_Pgamma): the full gamma rows m0,
// m0+1, t-1, t (x kept per mode, synthesised by a small inverse GEMM) and, on
// every row, u at q_lo-1, q_lo and their mirrors, i.e. the synthesis sums
//   sum_c x_m(c) S(c, q_lo-2 + base) and sum_c x_m(c) S(c, q_lo-1 + base)
// (real and imaginary parts: four values per row and parity block).
//
// Schedule: one wavefront per (64 L consecutive folded mode columns, column b);
// lane i sweeps the L columns c0 = wave base + i L .. c0 + L - 1 side by side
// (independent recurrences for latency, one row of factors per load), so each
// 64-column block of the fold (one parity) is a group of 64/L lanes.  The
// forward elimination keeps y only at the end of every K-row segment
// (checkpoints in HBM); the back substitution recomputes a segment's y from the
// checkpoint before it, walks back through it, and adds each row's four
// synthesis products over the lane's L columns; the group then reduces the 4 K
// sums of the segment across its lanes (a reduce-scatter: permlane swaps for
// the lane bits 32 and 16, DPP row permutations below) and writes them.
// Segments holding no special row (all but the first and the last one or two)
// take a path without the special-row tests.
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

#include "mdp_internal.h"

namespace mdp {
namespace {

template <class P>
__device__ inline const __attribute__((address_space(1))) P* gview(const P* p) {
    return (const __attribute__((address_space(1))) P*)p;
}

// The job of global column b (jobs sorted by b0).
__device__ inline int find_fused_job(const FusedJob* __restrict__ jobs, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- cross-lane moves
// DPP controls (a row is 16 lanes): rotate a row by 8 (= lane xor 8), mirror each
// half row (lane i of 8 <-> 7 - i, flipping lane bit 2), quad permutations
// [2,3,0,1] (xor 2) and [1,0,3,2] (xor 1).
constexpr int kDppRor8 = 0x128;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppXor1 = 0xB1;

template <int CTRL>
__device__ inline float dpp_mov(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_mov(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// permlane swaps exchange the odd 16-lane rows of a with the even rows of b (16), or
// the upper 32 lanes of a with the lower 32 of b (32): afterwards a + b holds, in a
// lane with the swapped lane bit clear, the pair's sum of a, otherwise of b.
template <bool S32>
__device__ inline void lane_swap(unsigned& a, unsigned& b) {
    if constexpr (S32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}
template <bool S32>
__device__ inline void lane_swap(float& a, float& b) {
    unsigned x = __builtin_bit_cast(unsigned, a), y = __builtin_bit_cast(unsigned, b);
    lane_swap<S32>(x, y);
    a = __builtin_bit_cast(float, x);
    b = __builtin_bit_cast(float, y);
}
template <bool S32>
__device__ inline void lane_swap(double& a, double& b) {
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
    const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
    unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32), blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
    lane_swap<S32>(alo, blo);
    lane_swap<S32>(ahi, bhi);
    a = __builtin_bit_cast(double, ((unsigned long long)ahi << 32) | alo);
    b = __builtin_bit_cast(double, ((unsigned long long)bhi << 32) | blo);
}

// One level of a butterfly reduce-scatter: the values v[0..2H) of a lane and of its
// partner across one lane bit; the lane with that bit set keeps the upper half,
// the other the lower half, each summed over the pair, in v[0..H).
template <class T, int H, bool S32>
__device__ inline void level_swap(T* v) {
#pragma unroll
    for (int j = 0; j < H; ++j) {
        lane_swap<S32>(v[j], v[H + j]);
        v[j] = v[j] + v[H + j];
    }
}
template <class T, int H, int CTRL>
__device__ inline void level_dpp(T* v, bool hi) {
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const T keep = hi ? v[H + j] : v[j];
        const T send = hi ? v[j] : v[H + j];
        v[j] = keep + dpp_mov<CTRL>(send);
    }
}

// Sums of the 32 values v[0..32) of every lane over its group of 64/L lanes (the
// lanes of one 64-column block).  Afterwards lane i of the group holds the total
// of value index vidx in v[e] for e < NOUT:
//   L = 1: NOUT = 1, vidx = i >> 1 (lanes 2j, 2j+1 both hold value j);
//   L = 2: NOUT = 1, vidx = i;
//   L = 4: NOUT = 2, vidx = 2 i + e.
template <class T, int L>
struct GroupReduce {
    static constexpr int NOUT = (L == 4) ? 2 : 1;
    __device__ static inline void run(T* v, int lane) {
        if constexpr (L == 1) {
            level_swap<T, 16, true>(v);
            level_swap<T, 8, false>(v);
            level_dpp<T, 4, kDppRor8>(v, lane & 8);
            level_dpp<T, 2, kDppHalfMirror>(v, lane & 4);
            level_dpp<T, 1, kDppXor2>(v, lane & 2);
            v[0] = v[0] + dpp_mov<kDppXor1>(v[0]);
        } else if constexpr (L == 2) {
            level_swap<T, 16, false>(v);
            level_dpp<T, 8, kDppRor8>(v, lane & 8);
            level_dpp<T, 4, kDppHalfMirror>(v, lane & 4);
            level_dpp<T, 2, kDppXor2>(v, lane & 2);
            level_dpp<T, 1, kDppXor1>(v, lane & 1);
        } else {
            level_dpp<T, 16, kDppRor8>(v, lane & 8);
            level_dpp<T, 8, kDppHalfMirror>(v, lane & 4);
            level_dpp<T, 4, kDppXor2>(v, lane & 2);
            level_dpp<T, 2, kDppXor1>(v, lane & 1);
        }
    }
    __device__ static inline int vidx(int lane, int e) {
        if constexpr (L == 1) return (lane & 63) >> 1;
        else if constexpr (L == 2) return lane & 31;
        else return 2 * (lane & 15) + e;
    }
    __device__ static inline bool writer(int lane) { return L != 1 || (lane & 1) == 0; }
};

// ---------------------------------------------------------------- the sweep
template <class T, int L>
struct Lanes {
    typedef T V __attribute__((ext_vector_type(2 * L)));   // L complex (re, im) pairs
    typedef T R __attribute__((ext_vector_type(L)));       // L real values
};

// Grid: one workgroup (one wavefront) per (column, block of 64 L mode columns), the
// block index fastest, so that consecutive workgroups, which the dispatcher deals
// round-robin to the eight XCDs, keep one mode block per XCD when nwb divides 8 (the
// factor rows of a block then stay in that XCD's L2).
template <class T, int L>
__global__ void __launch_bounds__(64) proj_sweep_kernel(const FusedJob* __restrict__ jobs, int njobs, int nwb) {
    constexpr int K = FUSED_K;
    static_assert(K == 8, "a segment is reduced as 8 rows x 4 products");
    typedef typename Lanes<T, L>::V V;
    typedef typename Lanes<T, L>::R Rv;
    typedef T T2 __attribute__((ext_vector_type(2)));
    const int gcol = blockIdx.x / nwb, wblk = blockIdx.x - gcol * nwb;
    const FusedJob& J = jobs[find_fused_job(jobs, njobs, gcol)];
    const int W = J.f.W, P1 = J.f.P1;
    const int wbase = wblk * 64 * L;
    if (wbase >= W) return;   // a job narrower than the launch (uniform over the wavefront)
    const int lane = threadIdx.x;
    const int c0 = wbase + lane * L;
    const bool live = c0 < W;              // lanes past W (a last wavefront of 64 columns when L > 1)
    const int cc = live ? c0 : 0;          // read column 0 there; nothing of theirs is written
    const bool odd = cc < P1;              // uniform over the lane's L columns (P1 is a multiple of 64)
    const int base = odd ? 0 : P1;
    const int n = J.f.n;
    const int m_lo = J.src.m_lo, m_hi = J.src.m_hi, q_lo = J.src.q_lo;
    const int m0 = m_lo - 1, t = m_hi + 1;
    const int nseg = J.nseg;
    const int b = gcol - J.b0;
    const long LW = W;

    const T* __restrict__ Sf = reinterpret_cast<const T*>(J.Sf);
    const T* __restrict__ Si = reinterpret_cast<const T*>(J.Si);
    const T* __restrict__ colc = reinterpret_cast<const T*>(J.colc);
    // factor rows: uniform row bases, the lane's vector at the 32-bit index lv (a row holds W / L
    // lane vectors), so that loads take a scalar base and a 32-bit lane offset
    const auto lf = gview(reinterpret_cast<const V*>(J.lf));
    const auto rf = gview(reinterpret_cast<const V*>(J.rf));
    const T* __restrict__ tf = reinterpret_cast<const T*>(J.tf);
    const int rowv = W / L;
    const unsigned lv = (unsigned)(cc / L);
    // the column's ring table: per row the pair (gA, gB) of its parity block
    const auto ring = gview(reinterpret_cast<const T2*>(reinterpret_cast<const T*>(J.gc) + (long)b * (n + 1) * 4));
    const unsigned rpar = odd ? 0u : 1u;
    const T* __restrict__ spec_hat = reinterpret_cast<const T*>(J.spec_hat) + (long)b * 4 * LW + cc;
    T* __restrict__ ck = reinterpret_cast<T*>(J.ckpt) + (long)b * nseg * 2 * LW + cc;
    T* __restrict__ xs = reinterpret_cast<T*>(J.xs) + (long)b * 8 * LW + cc;
    const int blk = (wbase >> 6) + lane / (64 / L);   // this lane group's 64-column block
    T* __restrict__ th = reinterpret_cast<T*>(J.thin) + ((long)b * (W >> 6) + blk) * ((long)nseg * K) * 4;

    // per-column constants: the transform of the two ring entries, the synthesis at
    // q_lo-1 and q_lo, the interior off-diagonal, the twisted pivot of row t
    T s1[L], s2[L], t1[L], t2[L], a[L], twr[L], twi[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int c = cc + l;
        s1[l] = Sf[(long)(base + q_lo - 1) * LW + c];
        s2[l] = Sf[(long)(base + q_lo) * LW + c];
        t1[l] = live ? Si[(long)c * LW + base + q_lo - 2] : T(0);
        t2[l] = live ? Si[(long)c * LW + base + q_lo - 1] : T(0);
        a[l] = colc[c];
        twr[l] = tf[2 * ((long)t * LW + c)];
        twi[l] = tf[2 * ((long)t * LW + c) + 1];
    }
    // special input row of m: 0..3, or -1 (uniform)
    auto special_in = [&](int m) -> int {
        return (m == m_lo) ? 0 : (m == m_lo + 1) ? 1 : (m == m_hi - 1) ? 2 : (m == m_hi) ? 3 : -1;
    };
    auto special_out = [&](int m) -> int {
        return (m == m0) ? 0 : (m == m0 + 1) ? 1 : (m == t - 1) ? 2 : (m == t) ? 3 : -1;
    };
    // a segment holding a special row (the first, and those reaching row t - 2)
    auto general = [&](int s) { return s == 0 || m0 + s * K + K - 1 >= t - 2; };

    // one elimination step of row m (rows past t are clamped to t by the caller)
    auto eliminate = [&](auto gen_tag, int m, T* yr, T* yi) {
        constexpr bool GEN = decltype(gen_tag)::value;
        const T2 g = ring[(long)m * 2 + rpar];
        const V fl = (lf + (long)m * rowv)[lv];
        T sp[L];
#pragma unroll
        for (int l = 0; l < L; ++l) sp[l] = T(0);
        if constexpr (GEN) {
            const int si = special_in(m);
            if (si >= 0) {
                const Rv v = *reinterpret_cast<const Rv*>(spec_hat + (long)si * LW);
#pragma unroll
                for (int l = 0; l < L; ++l) sp[l] = v[l];
            }
        }
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const T gh = fma(g.x, s1[l], fma(g.y, s2[l], sp[l]));
            const T lr = fl[2 * l], li = fl[2 * l + 1];
            const T nr = fma(-lr, yr[l], fma(li, yi[l], gh));
            const T ni = fma(-lr, yi[l], -(li * yr[l]));
            yr[l] = nr;
            yi[l] = ni;
        }
    };

    // forward elimination from row m0 (y_{m0-1} = 0), y kept at the end of every full segment
    {
        T yr[L], yi[L];
#pragma unroll
        for (int l = 0; l < L; ++l) yr[l] = yi[l] = T(0);
        auto fwd = [&](auto gen_tag, int s) {
#pragma unroll
            for (int i = 0; i < K; ++i) eliminate(gen_tag, m0 + s * K + i, yr, yi);
        };
        for (int s = 0; s < nseg - 1; ++s) {
            if (general(s)) fwd(std::true_type{}, s);
            else fwd(std::false_type{}, s);
            if (live) {
                Rv vr, vi;
#pragma unroll
                for (int l = 0; l < L; ++l) { vr[l] = yr[l]; vi[l] = yi[l]; }
                *reinterpret_cast<Rv*>(ck + (long)(2 * s) * LW) = vr;
                *reinterpret_cast<Rv*>(ck + (long)(2 * s + 1) * LW) = vi;
            }
        }
    }

    // back substitution segment by segment (x_{t+1} = 0, so the first row gives x_t = tw_t y_t)
    T xr[L], xi[L];
#pragma unroll
    for (int l = 0; l < L; ++l) xr[l] = xi[l] = T(0);
    auto bwd = [&](auto gen_tag, int s) {
        constexpr bool GEN = decltype(gen_tag)::value;
        const int mb = m0 + s * K;
        // y of the segment, recomputed from the checkpoint before it
        T vr[K][L], vi[K][L];
        {
            T yr[L], yi[L];
            if (s > 0) {
                const Rv pr = *reinterpret_cast<const Rv*>(ck + (long)(2 * s - 2) * LW);
                const Rv pi = *reinterpret_cast<const Rv*>(ck + (long)(2 * s - 1) * LW);
#pragma unroll
                for (int l = 0; l < L; ++l) { yr[l] = pr[l]; yi[l] = pi[l]; }
            } else {
#pragma unroll
                for (int l = 0; l < L; ++l) yr[l] = yi[l] = T(0);
            }
#pragma unroll
            for (int i = 0; i < K; ++i) {
                eliminate(gen_tag, GEN ? min(mb + i, t) : mb + i, yr, yi);
#pragma unroll
                for (int l = 0; l < L; ++l) { vr[i][l] = yr[l]; vi[i][l] = yi[l]; }
            }
        }
        // walk back through the segment: x_m = r_m (y_m - a x_{m+1}) (tw_t at row t), and the
        // row's synthesis products summed over the lane's columns
        T acc[4 * K];
#pragma unroll
        for (int i = K - 1; i >= 0; --i) {
            const int m = mb + i;
            acc[4 * i + 0] = acc[4 * i + 1] = acc[4 * i + 2] = acc[4 * i + 3] = T(0);
            if (GEN && m > t) continue;
            T rr[L], ri[L];
            if (GEN && m == t) {
#pragma unroll
                for (int l = 0; l < L; ++l) { rr[l] = twr[l]; ri[l] = twi[l]; }
            } else {
                const V fr = (rf + (long)m * rowv)[lv];
#pragma unroll
                for (int l = 0; l < L; ++l) { rr[l] = fr[2 * l]; ri[l] = fr[2 * l + 1]; }
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const T tr = fma(-a[l], xr[l], vr[i][l]);
                const T ti = fma(-a[l], xi[l], vi[i][l]);
                xr[l] = fma(rr[l], tr, -(ri[l] * ti));
                xi[l] = fma(rr[l], ti, ri[l] * tr);
                acc[4 * i + 0] = fma(xr[l], t1[l], acc[4 * i + 0]);
                acc[4 * i + 1] = fma(xi[l], t1[l], acc[4 * i + 1]);
                acc[4 * i + 2] = fma(xr[l], t2[l], acc[4 * i + 2]);
                acc[4 * i + 3] = fma(xi[l], t2[l], acc[4 * i + 3]);
            }
            if constexpr (GEN) {
                const int so = special_out(m);
                if (so >= 0 && live) {
                    Rv ore, oim;
#pragma unroll
                    for (int l = 0; l < L; ++l) { ore[l] = xr[l]; oim[l] = xi[l]; }
                    *reinterpret_cast<Rv*>(xs + (long)so * LW) = ore;
                    *reinterpret_cast<Rv*>(xs + (long)(4 + so) * LW) = oim;
                }
            }
        }
        GroupReduce<T, L>::run(acc, lane);
        if (blk < (W >> 6) && GroupReduce<T, L>::writer(lane)) {
#pragma unroll
            for (int e = 0; e < GroupReduce<T, L>::NOUT; ++e)
                th[(long)s * K * 4 + GroupReduce<T, L>::vidx(lane, e)] = acc[e];
        }
    };
    for (int s = nseg - 1; s >= 0; --s) {
        if (general(s)) bwd(std::true_type{}, s);
        else bwd(std::false_type{}, s);
    }
}

}  // namespace

namespace {

template <class T>
void launch_cols(int L, const FusedJob* jobs, int njobs, int total, int max_w, hipStream_t st) {
    const int nwb = (max_w + 64 * L - 1) / (64 * L);
    const long blocks = (long)total * nwb;
    if (blocks > 0x7fffffffL) throw Error(MDP_ERR_ARG, "too many projector columns for one launch");
    const dim3 grid((unsigned)blocks);
    if (L == 1)
        hipLaunchKernelGGL((proj_sweep_kernel<T, 1>), grid, dim3(64), 0, st, jobs, njobs, nwb);
    else if (L == 2)
        hipLaunchKernelGGL((proj_sweep_kernel<T, 2>), grid, dim3(64), 0, st, jobs, njobs, nwb);
    else if (L == 4)
        hipLaunchKernelGGL((proj_sweep_kernel<T, 4>), grid, dim3(64), 0, st, jobs, njobs, nwb);
    else
        throw Error(MDP_ERR_ARG, "columns per lane must be 1, 2 or 4");
    MDP_HIP(hipGetLastError());
}

// Autotuner of the sweep's schedule (mode columns per lane): per (precision, widest W,
// the batch's wavefront count at one column per lane within a factor of two), picked at
// first use by timing every candidate on the call's own data (one warm-up and two timed
// launches each, HIP events on the call's stream; the chosen one runs last, so the
// outputs are its own).  The schedules sum the synthesis products in different orders:
// results agree to rounding.
std::atomic<int> g_sweep_tune{0};
std::mutex g_sweep_mu;
std::map<std::tuple<int, int, int>, int> g_sweep_tuned;

}  // namespace

void set_sweep_autotune(int on) { g_sweep_tune.store(on ? 1 : 0); }

template <class T>
int launch_proj_sweep_jobs(const FusedJob* jobs, int njobs, int total, int max_w, long waves_one_col, int lanes_cols,
                           bool may_tune, hipStream_t st) {
    if (njobs <= 0 || total <= 0) return lanes_cols;
    if (!may_tune || !g_sweep_tune.load()) {
        launch_cols<T>(lanes_cols, jobs, njobs, total, max_w, st);
        return lanes_cols;
    }
    int lg = 0;
    while ((2L << lg) <= waves_one_col) ++lg;
    const auto key = std::make_tuple((int)sizeof(T), max_w, lg);
    {
        std::lock_guard<std::mutex> g(g_sweep_mu);
        auto it = g_sweep_tuned.find(key);
        if (it != g_sweep_tuned.end()) {
            launch_cols<T>(it->second, jobs, njobs, total, max_w, st);
            return it->second;
        }
    }
    hipEvent_t e0, e1;
    MDP_HIP(hipEventCreate(&e0));
    MDP_HIP(hipEventCreate(&e1));
    int best = lanes_cols;
    float best_ms = 1e30f;
    for (int L : {1, 2, 4}) {
        launch_cols<T>(L, jobs, njobs, total, max_w, st);
        MDP_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 2; ++r) launch_cols<T>(L, jobs, njobs, total, max_w, st);
        MDP_HIP(hipEventRecord(e1, st));
        MDP_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        MDP_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) { best_ms = ms; best = L; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> g(g_sweep_mu);
        g_sweep_tuned[key] = best;
    }
    launch_cols<T>(best, jobs, njobs, total, max_w, st);
    return best;
}
template int launch_proj_sweep_jobs<double>(const FusedJob*, int, int, int, long, int, bool, hipStream_t);
template int launch_proj_sweep_jobs<float>(const FusedJob*, int, int, int, long, int, bool, hipStream_t);

}  // namespace mdp
