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
// (twisted pivot tw_t).  With the LU factors r_m = 1/d'_m, the twisted pivot
// and the real interior off-diagonal a of the mode, the sweep runs in the
// unknowns scaled by a (q_m = a r_m y_m, x~_m = a x_m), so that one complex factor
// per row, ar_m = a r_m (a tw_t at row t), serves both directions:
//   q_m = ar_m (ghat_m - q_{m-1}),   x~_t = q_t,   x~_m = q_m - ar_m x~_{m+1},
// and x = x~ / a where x itself is needed.
// Q needs the solution on gamma only (eq. def_Pgamma): the full gamma rows m0,
// m0+1, t-1, t (x kept per mode, synthesised by a small inverse GEMM) and, on
// every row, u at q_lo-1, q_lo and their mirrors, i.e. the synthesis sums
//   sum_c x_m(c) S(c, q_lo-2 + base) and sum_c x_m(c) S(c, q_lo-1 + base)
// (real and imaginary parts: four values per row and parity block), formed as
// x~ times the synthesis weights over a.
//
// Schedule: one wavefront per (64 L consecutive folded mode columns, column b);
// lane i sweeps the L columns c0 = wave base + i L .. c0 + L - 1 side by side
// (independent recurrences for latency, one row of factors per load), so each
// 64-column block of the fold (one parity) is a group of 64/L lanes.  The
// forward elimination keeps q only at the end of every K-row segment
// (checkpoints in HBM); the back substitution recomputes a segment's q from the
// checkpoint before it, walks back through it, and adds each row's four
// synthesis products over the lane's L columns; the group then reduces the 4 K
// sums of the segment across its lanes (a reduce-scatter: permlane swaps for
// the lane bits 32 and 16, DPP row permutations below) and writes them (at two
// columns per lane, the wavefront's two blocks summed first when they share a
// parity).  The factor rows of a segment reach LDS by direct global-to-LDS
// transfers issued a segment ahead from wavefront-uniform row addresses.
// Segments holding no special row (all but the first and the last one or two)
// take a path without the special-row tests.  A special input row adds ar_m
// spec_hat_m to q_m after the ring step (the same sum, and no registers held for
// it across the step).
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

// LDS of one workgroup: two buffers (the segment being swept, the one being loaded) of
// the factor rows r_m of the workgroup's 64 L mode columns (interleaved complex, row
// after row), and of the ring rows (gA, gB of both parities) of its NW columns.
template <class T, int L>
struct SweepLds {
    static constexpr int K = FUSED_K;
    static constexpr int row_bytes = 64 * L * 2 * (int)sizeof(T);
    static constexpr int lane_bytes = L * 2 * (int)sizeof(T);   // a lane's factors of one row
    static constexpr int units = lane_bytes > 16 ? lane_bytes / 16 : 1;   // staged in 16-byte units
    static constexpr int fac_bytes = K * row_bytes;              // one buffer of factor rows
    static constexpr int ring_bytes_per_col = K * 4 * (int)sizeof(T);
    static constexpr int ring_bytes = 4 * ring_bytes_per_col;    // NW <= 4 columns
    static constexpr int bytes = 2 * (fac_bytes + ring_bytes);
    static_assert(ring_bytes <= 1024, "a segment's ring rows are staged by one 1 KB transfer");
    static_assert(fac_bytes % 1024 == 0, "factor rows are staged in 1 KB transfers");
    static_assert(lane_bytes <= 16 || units * 16 == lane_bytes, "a lane's factors are whole 16-byte units");
};

// A pointer into global memory with the address space explicit: loads and stores through it
// are global instructions, counted by the vector memory counter only (through a generic
// pointer they would be flat instructions, which also count against the LDS counter, so that
// every wait for an LDS read would also wait for them).
template <class X> using gptr = __attribute__((address_space(1))) X*;   // converted by C-style casts

__device__ inline void lds_dma16(const void* src, void* lds_dst) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                     (__attribute__((address_space(3))) void*)lds_dst, 16, 0, 0);
}

// Grid: one workgroup of NW wavefronts per (group of NW consecutive columns of one job,
// block of 64 L mode columns), the block index fastest, so that consecutive
// workgroups, which the dispatcher deals round-robin to the eight XCDs, keep one mode
// block per XCD when nwb divides 8 (its factor rows then stay in that XCD's L2).
// The NW wavefronts sweep their own columns through the same mode columns in step:
// per K-row segment they read the factor rows from LDS, which the workgroup loads
// one segment ahead with direct global-to-LDS transfers (one load of a factor row
// serves NW columns; the only global loads a segment waits for were issued a
// segment earlier).  A wavefront without a column (the job's last group) sweeps
// its group's last column again and writes nothing.
template <class T, int L>
__global__ void __launch_bounds__(256) proj_sweep_kernel(const FusedJob* __restrict__ jobs, int njobs, int nwb,
                                                          int lg_nw) {
    constexpr int K = FUSED_K;
    static_assert(K == 8, "a segment is reduced as 8 rows x 4 products");
    typedef SweepLds<T, L> S;
    typedef typename Lanes<T, L>::V V;
    typedef typename Lanes<T, L>::R Rv;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const int NW = 1 << lg_nw;
    const int grp = blockIdx.x / nwb, wblk = blockIdx.x - grp * nwb;
    int jlo = 0, jhi = njobs - 1;   // the job holding column group grp (jobs sorted by g0)
    while (jlo < jhi) {
        const int mid = (jlo + jhi + 1) >> 1;
        if (jobs[mid].g0[lg_nw] <= grp) jlo = mid;
        else jhi = mid - 1;
    }
    const FusedJob& J = jobs[jlo];
    const int W = J.f.W, P1 = J.f.P1;
    const int wbase = wblk * 64 * L;
    if (wbase >= W) return;   // a job narrower than the launch (uniform over the workgroup)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int bfirst = (grp - J.g0[lg_nw]) * NW;     // the group's first column (job-local)
    // the job's column count in a register: read through J inside the loops it would be
    // reloaded after every global store (which might alias the job table), and a scalar load
    // pending there makes every wait for an LDS read a wait for all of them
    const int R = J.R;
    const bool has_col = bfirst + wave < R;
    const int b = min(bfirst + wave, R - 1);
    const int c0 = wbase + lane * L;
    const bool live = c0 < W;              // lanes past W (a last wavefront of 64 columns when L > 1)
    const bool writes = live && has_col;
    const int cc = live ? c0 : 0;          // read column 0 there; nothing of theirs is written
    const bool odd = cc < P1;              // uniform over the lane's L columns (P1 is a multiple of 64)
    const int base = odd ? 0 : P1;
    const int n = J.f.n;
    const int m_lo = J.src.m_lo, m_hi = J.src.m_hi, q_lo = J.src.q_lo;
    const int m0 = m_lo - 1, t = m_hi + 1;
    const int nseg = J.nseg;
    const long LW = W;

    const gptr<const T> Sf = (gptr<const T>)(J.Sf);
    const gptr<const T> Si = (gptr<const T>)(J.Si);
    const gptr<const T> colc = (gptr<const T>)(J.colc);
    const T* __restrict__ tf = reinterpret_cast<const T*>(J.tf);
    const char* __restrict__ rtab = reinterpret_cast<const char*>(J.rf) + (long)wbase * 2 * sizeof(T);
    const char* __restrict__ twrow = reinterpret_cast<const char*>(J.tf) + ((long)t * LW + wbase) * 2 * sizeof(T);
    const char* __restrict__ gring = reinterpret_cast<const char*>(J.gc);
    const gptr<const T> spec_hat = (gptr<const T>)(J.spec_hat) + (long)b * 4 * LW + cc;
    const gptr<T> ck = (gptr<T>)(J.ckpt) + (long)b * nseg * 2 * LW + cc;
    const gptr<T> xs = (gptr<T>)(J.xs) + (long)b * 8 * LW + cc;
    const int blk = (wbase >> 6) + lane / (64 / L);   // this lane group's 64-column block
    const gptr<T> th = (gptr<T>)(J.thin) + ((long)b * (W >> 6) + blk) * ((long)nseg * K) * 4;

    // per-column constants: the transform of the two ring entries, the synthesis weights at
    // q_lo-1 and q_lo over the interior off-diagonal a, and 1/a (zero on padding columns)
    T s1[L], s2[L], t1[L], t2[L], ai[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int c = cc + l;
        const T a = colc[c];
        ai[l] = a != T(0) ? T(1) / a : T(0);
        s1[l] = Sf[(long)(base + q_lo - 1) * LW + c];
        s2[l] = Sf[(long)(base + q_lo) * LW + c];
        t1[l] = live ? Si[(long)c * LW + base + q_lo - 2] * ai[l] : T(0);
        t2[l] = live ? Si[(long)c * LW + base + q_lo - 1] * ai[l] : T(0);
    }
    auto special_in = [&](int m) -> int {
        return (m == m_lo) ? 0 : (m == m_lo + 1) ? 1 : (m == m_hi - 1) ? 2 : (m == m_hi) ? 3 : -1;
    };
    auto special_out = [&](int m) -> int {
        return (m == m0) ? 0 : (m == m0 + 1) ? 1 : (m == t - 1) ? 2 : (m == t) ? 3 : -1;
    };
    // a segment holding a special row (the first, and those reaching row t - 2)
    auto general = [&](int s) { return s == 0 || m0 + s * K + K - 1 >= t - 2; };

    // staging of segment s into buffer sb: the factor rows r_m, m = mb..mb+K-1, of the
    // workgroup's mode columns in 1 KB transfers shared out over the wavefronts (at row t,
    // and the rows past it, the twisted pivot tw_t: the elimination step p = r y then gives
    // x_t = tw_t y_t there, and the rows past t are not used), and the ring rows of the NW
    // columns in one transfer by wavefront 0
    char* const fac_buf = lds;
    char* const ring_buf = lds + 2 * S::fac_bytes;
    // A row whose lane share exceeds 16 bytes is staged unit-major: with U 16-byte units per lane,
    // LDS unit u * 64 + j of a row holds lane j's unit u, so that each of a lane's U reads below is
    // contiguous over the wavefront (no LDS bank conflicts); shares of 8 or 16 bytes are read
    // contiguously as they are.
    constexpr int U = S::units;
    constexpr bool unit_major = S::lane_bytes > 16;
    // With rows of 1 KB or more, transfer ch is piece cr = ch mod (row_bytes / 1 KB) of row ch / (row_bytes
    // / 1 KB): its row and piece are the same for the whole wavefront, so the source is a wavefront-uniform
    // row address (kept in scalar registers) plus a per-lane offset fixed for the whole sweep: LDS unit
    // 64 cr + lane holds global unit lane U + cr (unit-major) or 64 cr + lane.
    const int lane_off = unit_major ? lane * U * 16 : lane * 16;
    auto stage = [&](int s, int sb) {
        const int mb = m0 + s * K;
        char* fdst = fac_buf + sb * S::fac_bytes;
        if constexpr (S::row_bytes >= 1024) {
            constexpr int CPR = S::row_bytes / 1024, piece = unit_major ? 16 : 1024;
            for (int ch = wave; ch < S::fac_bytes / 1024; ch += NW) {
                const int i = ch / CPR, cr = ch - i * CPR;
                const int m = mb + i;
                const char* row = (m < t ? rtab + (long)m * LW * 2 * sizeof(T) : twrow) + cr * piece;
                lds_dma16(row + lane_off, fdst + ch * 1024);
            }
        } else {
            for (int ch = wave; ch < S::fac_bytes / 1024; ch += NW) {
                const int o = ch * 1024 + lane * 16;
                const int i = o / S::row_bytes, p = (o - i * S::row_bytes) / 16;
                const int cb = unit_major ? ((p & 63) * U + (p >> 6)) * 16 : p * 16;   // the global unit it holds
                const int m = mb + i;
                lds_dma16((m < t ? rtab + (long)m * LW * 2 * sizeof(T) : twrow) + cb, fdst + ch * 1024);
            }
        }
        if (wave == 0) {
            const int o = lane * 16;
            if (o < NW * S::ring_bytes_per_col) {
                const int wv = o / S::ring_bytes_per_col, rem = o - wv * S::ring_bytes_per_col;
                const int i = rem / (4 * (int)sizeof(T)), part = rem - i * 4 * (int)sizeof(T);
                const int bw = min(bfirst + wv, R - 1);
                const int m = min(mb + i, t);
                lds_dma16(gring + (((long)bw * (n + 1) + m) * 4) * sizeof(T) + part, ring_buf + sb * S::ring_bytes);
            }
        }
    };
    // factor row i of buffer sb for the lane's columns, and the column's ring pair of row i
    auto fac = [&](int sb, int i) -> V {
        if constexpr (!unit_major)
            return *reinterpret_cast<const V*>(fac_buf + sb * S::fac_bytes + i * S::row_bytes + lane * S::lane_bytes);
        typedef T Unit __attribute__((ext_vector_type(16 / sizeof(T))));
        const char* row = fac_buf + sb * S::fac_bytes + i * S::row_bytes + lane * 16;
        V f;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const Unit x = *reinterpret_cast<const Unit*>(row + u * 64 * 16);
#pragma unroll
            for (int e = 0; e < (int)(16 / sizeof(T)); ++e) f[u * (16 / sizeof(T)) + e] = x[e];
        }
        return f;
    };
    auto ring = [&](int sb, int i, T& gA, T& gB) {
        const T* r = reinterpret_cast<const T*>(ring_buf + sb * S::ring_bytes + wave * S::ring_bytes_per_col) +
                     i * 4 + (odd ? 0 : 2);
        gA = r[0];
        gB = r[1];
    };
    // one step of the forward elimination at row m: q = ar (ghat - q_prev) (the staged ar is
    // a tw_t at row t, so q is x~_t there), in place in (qr, qi); a special input row then adds
    // ar spec_hat (a uniform branch: read only on those four rows)
    auto step = [&](auto gen_tag, int sb, int i, int m, T* qr, T* qi) {
        constexpr bool GEN = decltype(gen_tag)::value;
        T gA, gB;
        ring(sb, i, gA, gB);
        const V f = fac(sb, i);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const T yr = fma(gA, s1[l], fma(gB, s2[l], -qr[l]));   // y = ghat - q_prev, yi = -qi
            const T rr = f[2 * l], ri = f[2 * l + 1];
            const T nr = fma(rr, yr, ri * qi[l]);
            qi[l] = fma(ri, yr, -(rr * qi[l]));
            qr[l] = nr;
        }
        if constexpr (GEN) {
            const int si = special_in(m);
            if (si >= 0) {
                const Rv v = *(gptr<const Rv>)(spec_hat + (long)si * LW);
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    qr[l] = fma(f[2 * l], v[l], qr[l]);
                    qi[l] = fma(f[2 * l + 1], v[l], qi[l]);
                }
            }
        }
    };

    // forward elimination from row m0 (q_{m0-1} = 0), q kept at the end of every full segment
    stage(0, 0);
    __syncthreads();
    Rv ckr, cki;   // the last checkpoint (q at the end of segment nseg - 2)
    {
        T qr[L], qi[L];
#pragma unroll
        for (int l = 0; l < L; ++l) qr[l] = qi[l] = T(0);
        // the checkpoint of segment s is stored after the barrier that ends it (the barrier waits
        // for every outstanding memory operation of the wavefront: a store issued just before it
        // would hold it for the store's whole latency)
        auto store_ck = [&](int s) {
            if (writes) {
                *(gptr<Rv>)(ck + (long)(2 * s) * LW) = ckr;
                *(gptr<Rv>)(ck + (long)(2 * s + 1) * LW) = cki;
            }
        };
        for (int s = 0; s < nseg - 1; ++s) {
            const int sb = s & 1;
            stage(s + 1, sb ^ 1);
            if (s > 0) store_ck(s - 1);
            auto fwd = [&](auto gen_tag) {
#pragma unroll
                for (int i = 0; i < K; ++i) step(gen_tag, sb, i, m0 + s * K + i, qr, qi);
            };
            if (general(s)) fwd(std::true_type{});
            else fwd(std::false_type{});
#pragma unroll
            for (int l = 0; l < L; ++l) { ckr[l] = qr[l]; cki[l] = qi[l]; }
            __syncthreads();   // buffer sb free, segment s+1 staged (the barrier waits for the transfers)
        }
        if (nseg >= 2) store_ck(nseg - 2);
    }

    // back substitution segment by segment (x~_{t+1} = 0, so row t gives x~_t = q_t):
    // recompute the segment's q from the checkpoint before it, then walk back through it,
    // x~_m = q_m - ar_m x~_{m+1}, adding each row's synthesis products
    T xr[L], xi[L];
#pragma unroll
    for (int l = 0; l < L; ++l) xr[l] = xi[l] = T(0);
    Rv cqr, cqi;   // the checkpoint the next segment starts from, loaded a segment ahead
    if (nseg >= 2) {   // the first one still in registers
        cqr = ckr;
        cqi = cki;
    }
    T thv[GroupReduce<T, L>::NOUT];   // the lane's reduced synthesis sums of the last segment
    // With two columns per lane a wavefront covers two 64-column blocks; unless they straddle
    // the parity boundary P1 (both odd or both even modes, or the second past W and all zero)
    // the wavefront adds their sums and writes them to the first block's slot only.
    const bool pair = L == 2 && wbase + 64 != P1;
    auto store_thin = [&](int s) {
        if (has_col && blk < (W >> 6) && GroupReduce<T, L>::writer(lane) && (!pair || lane < 32)) {
#pragma unroll
            for (int e = 0; e < GroupReduce<T, L>::NOUT; ++e) th[(long)s * K * 4 + GroupReduce<T, L>::vidx(lane, e)] = thv[e];
        }
    };
    for (int s = nseg - 1; s >= 0; --s) {
        const int sb = s & 1;   // segment nseg-1 was staged by the forward pass's last step
        T qr[L], qi[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            qr[l] = s > 0 ? cqr[l] : T(0);
            qi[l] = s > 0 ? cqi[l] : T(0);
        }
        if (s > 0) stage(s - 1, sb ^ 1);
        if (s > 1) {
            cqr = *(gptr<const Rv>)(ck + (long)(2 * s - 4) * LW);
            cqi = *(gptr<const Rv>)(ck + (long)(2 * s - 3) * LW);
        }
        auto bwd = [&](auto gen_tag) {
            constexpr bool GEN = decltype(gen_tag)::value;
            const int mb = m0 + s * K;
            T vr[K][L], vi[K][L];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                step(gen_tag, sb, i, mb + i, qr, qi);
#pragma unroll
                for (int l = 0; l < L; ++l) { vr[i][l] = qr[l]; vi[i][l] = qi[l]; }
            }
            // read the factor rows again below rather than keep them in registers across the two
            // walks (a compiler-level memory barrier; no instruction is emitted)
            asm volatile("" ::: "memory");
            T acc[4 * K];
#pragma unroll
            for (int i = K - 1; i >= 0; --i) {
                const int m = mb + i;
                acc[4 * i + 0] = acc[4 * i + 1] = acc[4 * i + 2] = acc[4 * i + 3] = T(0);
                if (GEN && m > t) continue;
                const V f = fac(sb, i);
#pragma unroll
                for (int l = 0; l < L; ++l) {   // x~ = q - ar x~_next
                    const T rr = f[2 * l], ri = f[2 * l + 1];
                    const T nr = fma(-rr, xr[l], fma(ri, xi[l], vr[i][l]));
                    xi[l] = fma(-rr, xi[l], fma(-ri, xr[l], vi[i][l]));
                    xr[l] = nr;
                    acc[4 * i + 0] = fma(xr[l], t1[l], acc[4 * i + 0]);
                    acc[4 * i + 1] = fma(xi[l], t1[l], acc[4 * i + 1]);
                    acc[4 * i + 2] = fma(xr[l], t2[l], acc[4 * i + 2]);
                    acc[4 * i + 3] = fma(xi[l], t2[l], acc[4 * i + 3]);
                }
                if constexpr (GEN) {
                    const int so = special_out(m);
                    if (so >= 0 && writes) {
                        Rv ore, oim;
#pragma unroll
                        for (int l = 0; l < L; ++l) { ore[l] = xr[l] * ai[l]; oim[l] = xi[l] * ai[l]; }
                        *(gptr<Rv>)(xs + (long)so * LW) = ore;
                        *(gptr<Rv>)(xs + (long)(4 + so) * LW) = oim;
                    }
                }
            }
            GroupReduce<T, L>::run(acc, lane);
            if constexpr (L == 2) {
                if (pair) {   // lanes j and j + 32 hold the same sum of the two blocks
                    T hi = acc[0];
                    lane_swap<true>(acc[0], hi);
                    acc[0] += hi;
                }
            }
#pragma unroll
            for (int e = 0; e < GroupReduce<T, L>::NOUT; ++e) thv[e] = acc[e];
        };
        if (general(s)) bwd(std::true_type{});
        else bwd(std::false_type{});
        __syncthreads();   // buffer sb free, segment s-1 staged
        store_thin(s);     // after the barrier, like the checkpoints
    }
}

}  // namespace

namespace {

template <class T, int L>
void launch_cl(const FusedJob* jobs, int njobs, long groups, int nwb, int lg_nw, hipStream_t st) {
    const long blocks = groups * nwb;
    if (blocks > 0x7fffffffL) throw Error(MDP_ERR_ARG, "too many projector columns for one launch");
    constexpr int lds_bytes = SweepLds<T, L>::bytes;
    const void* fn = reinterpret_cast<const void*>(&proj_sweep_kernel<T, L>);
    static const bool lds_set = [fn] {   // more than 64 KB of dynamic LDS must be allowed explicitly
        if (lds_bytes > 65536) MDP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes));
        return true;
    }();
    (void)lds_set;
    hipLaunchKernelGGL((proj_sweep_kernel<T, L>), dim3((unsigned)blocks), dim3(64 << lg_nw), lds_bytes, st, jobs, njobs,
                       nwb, lg_nw);
}

// Wavefronts per workgroup for L columns per lane: four (one staged factor row serves four
// columns) while that leaves at least four workgroups per CU of the chip (256 CUs), else
// fewer (small batches: the workgroups' barriers would keep too few wavefronts busy).
int lg_waves_per_group(long total, int max_w, int L) {
    const long waves = total * ((max_w + 64 * L - 1) / (64 * L));
    return waves >= 4L * 1024 ? 2 : waves >= 2L * 1024 ? 1 : 0;
}

// groups[lg] = number of column groups of 1 << lg columns over all jobs (the jobs' g0 tables)
template <class T>
void launch_cols(int L, const FusedJob* jobs, int njobs, int total, const long* groups, int max_w, hipStream_t st) {
    const int lg_nw = lg_waves_per_group(total, max_w, L);
    const int nwb = (max_w + 64 * L - 1) / (64 * L);
    if (L == 1) launch_cl<T, 1>(jobs, njobs, groups[lg_nw], nwb, lg_nw, st);
    else if (L == 2) launch_cl<T, 2>(jobs, njobs, groups[lg_nw], nwb, lg_nw, st);
    else if (L == 4) launch_cl<T, 4>(jobs, njobs, groups[lg_nw], nwb, lg_nw, st);
    else throw Error(MDP_ERR_ARG, "columns per lane must be 1, 2 or 4");
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
int launch_proj_sweep_jobs(const FusedJob* jobs, int njobs, int total, const long* groups, int max_w,
                           long waves_one_col, int lanes_cols, bool may_tune, hipStream_t st) {
    if (njobs <= 0 || total <= 0) return lanes_cols;
    if (!may_tune || !g_sweep_tune.load()) {
        launch_cols<T>(lanes_cols, jobs, njobs, total, groups, max_w, st);
        return lanes_cols;
    }
    int lg = 0;
    while ((2L << lg) <= waves_one_col) ++lg;
    const auto key = std::make_tuple((int)sizeof(T), max_w, lg);
    {
        std::lock_guard<std::mutex> g(g_sweep_mu);
        auto it = g_sweep_tuned.find(key);
        if (it != g_sweep_tuned.end()) {
            launch_cols<T>(it->second, jobs, njobs, total, groups, max_w, st);
            return it->second;
        }
    }
    hipEvent_t e0, e1;
    MDP_HIP(hipEventCreate(&e0));
    MDP_HIP(hipEventCreate(&e1));
    int best = lanes_cols;
    float best_ms = 1e30f;
    for (int L : {1, 2, 4}) {
        launch_cols<T>(L, jobs, njobs, total, groups, max_w, st);
        MDP_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 2; ++r) launch_cols<T>(L, jobs, njobs, total, groups, max_w, st);
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
    launch_cols<T>(best, jobs, njobs, total, groups, max_w, st);
    return best;
}
template int launch_proj_sweep_jobs<double>(const FusedJob*, int, int, const long*, int, long, int, bool, hipStream_t);
template int launch_proj_sweep_jobs<float>(const FusedJob*, int, int, const long*, int, long, int, bool, hipStream_t);

}  // namespace mdp
