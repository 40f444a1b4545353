// Hand-written CDNA4 (gfx950) matrix-core GEMM used by the particle-particle
// term and the large contractions of sigma.
//
//   C[perm(m, n)] = alpha * sum_k opA(A)[m][k] * opB(B)[k][n] + beta * C[...]
//
// A is addressed as [m][k] (row-major, k fastest) unless transposed ([k][m]);
// B is addressed as [n][k] ("NT", k fastest) unless given as [k][n].  Both
// operands are staged through LDS as [row][k] tiles; the k-fastest forms load
// 16-byte vectors straight into that layout, the other forms transpose while
// writing LDS.  Accumulation is in the MFMA accumulator type (FP64 for FP64,
// FP32 for FP32 and BF16 inputs).
//
// Instruction shapes (one 64-lane wave, a 16x16 output block per instruction):
//   FP64  v_mfma_f64_16x16x4f64       k = 4 per instruction
//   FP32  v_mfma_f32_16x16x4f32       k = 4
//   BF16  v_mfma_f32_16x16x32_bf16    k = 32 (8 per lane)
// Lane l holds operand rows (l mod 16) and a k-slice chosen by l / 16; result
// register r holds column (l mod 16) and row 4*(l/16)+r (FP32 accumulators)
// or row (l/16)+4r (FP64 accumulators), r = 0..3.  Since only
// the sum over k matters, each lane's k-slice within a BK tile is a contiguous
// run of BK/4 elements (32 bytes), read from LDS with two 16-byte loads.
//
// The output index map supports the permuted store of the rebuilt
// four-index block: row m = (m1, m2) with m2 = m mod rsplit, column
// n = (n1, n2) with n2 = n mod csplit, and
//   C offset = m1*rs1 + m2*rs2 + n1*cs1 + n2*cs2 + batch*sC.
#pragma once

#include "mfma_gemm.hpp"

#include <algorithm>
#include <type_traits>

namespace adc {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    using acc_t = double;
    using accv = d4v;
    static constexpr int BK = 16;       // k per LDS tile (4 per lane: 32 bytes)
    static constexpr int KSTEP = 4;     // k per instruction
    // result register r of lane l holds row (l/16) + 4r (rows interleaved)
    static __device__ __forceinline__ int row(int lg, int r) { return lg + 4 * r; }
    static __device__ __forceinline__ accv step(const uint4* la, const uint4* lb, int s, accv c) {
        double a = reinterpret_cast<const double*>(la)[s];
        double b = reinterpret_cast<const double*>(lb)[s];
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <>
struct Mfma<float> {
    using acc_t = float;
    using accv = f4v;
    static constexpr int BK = 32;       // 8 per lane
    static constexpr int KSTEP = 4;
    // result register r of lane l holds row 4(l/16) + r
    static __device__ __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
    static __device__ __forceinline__ accv step(const uint4* la, const uint4* lb, int s, accv c) {
        float a = reinterpret_cast<const float*>(la)[s];
        float b = reinterpret_cast<const float*>(lb)[s];
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <>
struct Mfma<bf16_t> {
    using acc_t = float;
    using accv = f4v;
    static constexpr int BK = 64;       // 16 per lane
    static constexpr int KSTEP = 32;
    static __device__ __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
    static __device__ __forceinline__ accv step(const uint4* la, const uint4* lb, int s, accv c) {
        bf8v a = __builtin_bit_cast(bf8v, la[s]);
        bf8v b = __builtin_bit_cast(bf8v, lb[s]);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

template <typename TO, typename TA>
__device__ __forceinline__ TO to_out(TA v) {
    return (TO)v;
}

// A 16-byte chunk of VW compute-type elements read from storage type TI
// (the same type, or FP32 rounded to BF16 on the way into LDS).
template <typename TI, typename TC>
struct Chunk {
    static constexpr int VW = 16 / sizeof(TC);
    static __device__ __forceinline__ uint4 vec(const TI* p) {
        if constexpr (sizeof(TI) == sizeof(TC)) {
            return *reinterpret_cast<const uint4*>(p);
        } else {
            static_assert(sizeof(TI) == 4 && sizeof(TC) == 2, "FP32 -> BF16 only");
            TC v[VW];
#pragma unroll
            for (int h = 0; h < VW / 4; ++h) {
                float4 f = reinterpret_cast<const float4*>(p)[h];
                v[4 * h + 0] = (TC)f.x;
                v[4 * h + 1] = (TC)f.y;
                v[4 * h + 2] = (TC)f.z;
                v[4 * h + 3] = (TC)f.w;
            }
            return __builtin_bit_cast(uint4, v);
        }
    }
};

// Origin (m0, n0) of this workgroup's BM x BN output tile.  Workgroups are
// dealt round-robin to the 8 XCDs, so the linear id is regrouped to give each
// XCD a contiguous run of tiles, walked in column groups of 8 row tiles
// (operand reuse in that XCD's L2).
template <int BM, int BN>
__device__ __forceinline__ void tile_origin(const GemmShape& g, long long& m0, long long& n0) {
    const long long ntn = (g.N + BN - 1) / BN, ntm = (g.M + BM - 1) / BM;
    // hardware id h goes to XCD h mod 8; XCD x takes the logical ids
    // [x*q + min(x, r), ...) of length q + (x < r), q = nwg / 8, r = nwg mod 8
    long long pid = blockIdx.x;
    const long long nwg = (long long)gridDim.x;
    {
        const long long x = pid & 7, k = pid >> 3, q = nwg >> 3, r = nwg & 7;
        pid = x * q + (x < r ? x : r) + k;
    }
    const long long GROUP = 8;
    const long long per_group = GROUP * ntn;
    const long long grp = pid / per_group;
    const long long first_m = grp * GROUP;
    const long long gsz = std::min(ntm - first_m, GROUP);
    const long long tmi = first_m + (pid % per_group) % gsz;
    const long long tni = (pid % per_group) / gsz;
    m0 = tmi * BM;
    n0 = tni * BN;
}

// Element offsets of this workgroup's batch entry (grid z, two levels) in the
// operands and the result.
struct BatchOff {
    long long a, b, c;
};
__device__ __forceinline__ BatchOff batch_offsets(const GemmShape& g) {
    const long long bz = g.z0 + blockIdx.z;
    const long long b1 = bz / g.n2, b2 = bz - b1 * g.n2;
    return {b1 * g.sA + b2 * g.sA2, b1 * g.sB + b2 * g.sB2, b1 * g.sC + b2 * g.sC2};
}

// Store of one wave's WM x WN block of accumulators, whose first output row
// and column are (mw, nw).  The block is staged in LDS at `stage` (alpha
// applied), in NPASS passes over column slices, and stored back through the
// output index map in runs of 4 consecutive columns: one vector store per run
// when the run is contiguous and aligned in the map, element stores otherwise.
// Every wave of the workgroup calls it (it synchronises the workgroup).
template <typename T, typename TO, int WM, int WN, int NPASS>
__device__ __forceinline__ void store_tile(typename Mfma<T>::accv (&acc)[WM / 16][WN / 16],
                                           typename Mfma<T>::acc_t* stage, TO* __restrict__ C,
                                           const GemmShape& g, long long mw, long long nw,
                                           int lane, typename Mfma<T>::acc_t alpha,
                                           typename Mfma<T>::acc_t beta) {
    using MT = Mfma<T>;
    using acc_t = typename MT::acc_t;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int PAD = 16 / (int)sizeof(acc_t);
    constexpr int WNP = WN / NPASS;          // columns per pass
    constexpr int TNP = TN / NPASS;          // 16-column blocks per pass
    constexpr int LDC = WNP + PAD;           // staged row (elements)
    constexpr int RUNS = WM * WNP / 4;       // runs of 4 per wave and pass
    static_assert(TN % NPASS == 0 && RUNS % 64 == 0, "epilogue tiling");
    typedef TO to4 __attribute__((ext_vector_type(4)));
    const int li = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
        __syncthreads();    // operand tiles (or the previous pass) no longer read
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int jj = 0; jj < TNP; ++jj)
                    stage[(i * 16 + MT::row(lg, r)) * LDC + jj * 16 + li] =
                        alpha * acc[i][p * TNP + jj][r];
        __syncthreads();
        // one run = 4 consecutive columns of one row; a lane keeps the same
        // columns across its runs (64 is a multiple of the runs per row), so
        // the column split is computed once per pass and the row split
        // advanced incrementally (no 64-bit division per run)
        constexpr int RPR = WNP / 4;              // runs per row
        static_assert(64 % RPR == 0, "epilogue: runs per row must divide 64");
        constexpr int RSTEP = 64 / RPR;           // rows between a lane's runs
        const int c4 = (lane % RPR) * 4;
        const long long n = nw + p * WNP + c4;
        const long long n1 = n / g.csplit, n2 = n - n1 * g.csplit;
        const bool nrun = n + 3 < g.N && g.cs2 == 1 && n2 + 3 < g.csplit;
        long long m = mw + lane / RPR;
        long long m1 = m / g.rsplit, m2 = m - m1 * g.rsplit;
        const long long coff = n1 * g.cs1 + n2 * g.cs2;
#pragma unroll 4
        for (int row = lane / RPR; row < WM; row += RSTEP) {
            if (m < g.M && n < g.N) {
                const acc_t* sv = stage + row * LDC + c4;
                TO* dst = C + m1 * g.rs1 + m2 * g.rs2 + coff;
                const bool run =
                    nrun && (reinterpret_cast<uintptr_t>(dst) % (4 * sizeof(TO))) == 0;
                if (run) {
                    to4 o;
                    if (beta != acc_t(0)) {
                        const to4 old = *reinterpret_cast<const to4*>(dst);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            o[e] = to_out<TO, acc_t>(sv[e] + beta * (acc_t)old[e]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) o[e] = to_out<TO, acc_t>(sv[e]);
                    }
                    *reinterpret_cast<to4*>(dst) = o;
                } else {
                    for (int e = 0; e < 4 && n + e < g.N; ++e) {
                        const long long ne = n + e, ne1 = ne / g.csplit, ne2 = ne - ne1 * g.csplit;
                        TO* de = C + m1 * g.rs1 + m2 * g.rs2 + ne1 * g.cs1 + ne2 * g.cs2;
                        acc_t v = sv[e];
                        if (beta != acc_t(0)) v += beta * (acc_t)(*de);
                        *de = to_out<TO, acc_t>(v);
                    }
                }
            }
            m += RSTEP;
            m2 += RSTEP;
            while (m2 >= g.rsplit) {
                m2 -= g.rsplit;
                ++m1;
            }
        }
    }
}

// One workgroup of 256 threads (4 waves) computes a BM x BN tile; each wave a
// WM x WN sub-tile of 16x16 instruction blocks.
// A workgroup of WGM x WGN waves computes a BM x BN tile, each wave a
// (BM/WGM) x (BN/WGN) block of 16x16 instruction tiles.  KIND only names the
// kernel for profiles (0 plain, 1 four-index rebuild, 2 particle-particle
// contraction); the code is the same.
template <typename TI, typename T, typename TO, int BM, int BN, int WGM, int WGN, bool TA, bool TB,
          int KIND>
__global__ void __launch_bounds__(64 * WGM * WGN)
k_gemm(const TI* __restrict__ A, const TI* __restrict__ B, TO* __restrict__ C, GemmShape g,
       typename Mfma<T>::acc_t alpha, typename Mfma<T>::acc_t beta) {
    using MT = Mfma<T>;
    using acc_t = typename MT::acc_t;
    using accv = typename MT::accv;
    constexpr int NT = 64 * WGM * WGN;               // threads
    constexpr int BK = MT::BK;
    constexpr int VW = 16 / sizeof(T);               // elements per 16-byte vector
    constexpr int LDK = BK + VW;                     // padded LDS row (elements)
    constexpr int WAVES_N = WGN;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int NSTEP = BK / MT::KSTEP;
    static_assert(TM >= 1 && TN >= 1, "tile too small");

    // operand tiles, double-buffered; reused by the epilogue to stage results
    __shared__ __attribute__((aligned(16))) T smem[2 * (BM + BN) * LDK];
    auto sA = [&](int b) -> T* { return smem + b * (BM * LDK); };
    auto sB = [&](int b) -> T* { return smem + 2 * BM * LDK + b * (BN * LDK); };

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    const int li = lane & 15, lg = lane >> 4;

    long long m0, n0;
    tile_origin<BM, BN>(g, m0, n0);
    {
        const BatchOff o = batch_offsets(g);
        A += o.a;
        B += o.b;
        C += o.c;
    }

    // ---- global -> register staging ------------------------------------
    // A chunk is 16 bytes of compute-type elements: VW consecutive k of one
    // row ([row][k] source) or VW consecutive rows of one k ([k][row] source).
    constexpr int CA = BM * BK / VW / NT;   // chunks per thread (A)
    constexpr int CB = BN * BK / VW / NT;
    static_assert(CA >= 1 && CB >= 1 && CA * NT * VW == BM * BK && CB * NT * VW == BN * BK,
                  "tile does not split into 16-byte chunks per thread");
    uint4 ra[CA], rb[CB];

    // 16-byte loads of a full k-tile (k0 + BK <= K) of an aligned operand.
    // Rows past the operand's extent only feed output rows (columns) that the
    // epilogue discards, so their addresses are clamped into the operand
    // instead of being checked: a [row][k] source reads its last row again, a
    // [k][row] source (ld a multiple of VW) reads the last VW entries of the
    // k-row.  Any tile of the grid runs this path.
    auto load_fast = [&](const TI* P, long long ld, auto trans_tag, long long R0, long long Rmax,
                         int R, uint4* r, int nchunk, long long k0) {
        constexpr bool TR = decltype(trans_tag)::value;
#pragma unroll
        for (int c = 0; c < nchunk; ++c) {
            const int id = tid + c * NT;
            if constexpr (!TR) {
                long long row = R0 + id / (BK / VW);
                row = row < Rmax ? row : Rmax - 1;
                const int kc = (id % (BK / VW)) * VW;
                r[c] = Chunk<TI, T>::vec(P + row * ld + k0 + kc);
            } else {
                const int kk = id / (R / VW);
                long long col = R0 + (id % (R / VW)) * VW;
                col = col <= ld - VW ? col : ld - VW;
                r[c] = Chunk<TI, T>::vec(P + (k0 + kk) * ld + col);
            }
        }
    };
    // element loads with bounds checks, branch-free: an out-of-range element
    // reads P[0] and is replaced by zero
    auto load_safe = [&](const TI* P, long long ld, auto trans_tag, long long R0, long long Rmax,
                         int R, uint4* r, int nchunk, long long k0) {
        constexpr bool TR = decltype(trans_tag)::value;
#pragma unroll
        for (int c = 0; c < nchunk; ++c) {
            const int id = tid + c * NT;
            T v[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                long long gr, gk;
                if constexpr (!TR) {
                    gr = R0 + id / (BK / VW);
                    gk = k0 + (id % (BK / VW)) * VW + e;
                } else {
                    gk = k0 + id / (R / VW);
                    gr = R0 + (id % (R / VW)) * VW + e;
                }
                const bool ok = gr < Rmax && gk < g.K;
                const long long off = TR ? gk * ld + gr : gr * ld + gk;
                const TI x = P[ok ? off : 0];
                v[e] = ok ? (T)x : T(0);
            }
            r[c] = __builtin_bit_cast(uint4, v);
        }
    };
    auto store = [&](T* S, auto trans_tag, int R, const uint4* r, int nchunk) {
        constexpr bool TR = decltype(trans_tag)::value;
#pragma unroll
        for (int c = 0; c < nchunk; ++c) {
            const int id = tid + c * NT;
            if constexpr (!TR) {
                const int row = id / (BK / VW), kc = (id % (BK / VW)) * VW;
                *reinterpret_cast<uint4*>(S + row * LDK + kc) = r[c];
            } else {
                const int kk = id / (R / VW), rc = (id % (R / VW)) * VW;
                T v[VW];
                *reinterpret_cast<uint4*>(v) = r[c];
#pragma unroll
                for (int e = 0; e < VW; ++e) S[(rc + e) * LDK + kk] = v[e];
            }
        }
    };
    using TrA = std::integral_constant<bool, TA>;
    using TrB = std::integral_constant<bool, !TB>;

    accv acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = accv{};

    auto compute = [&](int cur) {
        // fragments: each lane's contiguous k-run of BK/4 elements (32 bytes)
        if constexpr (sizeof(T) == 8) {
#pragma unroll
            for (int s = 0; s < NSTEP; ++s) {
                double fa[TM], fb[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    fa[i] = *reinterpret_cast<const double*>(
                        sA(cur) + (wm * WM + i * 16 + li) * LDK + lg * (BK / 4) + s);
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    fb[j] = *reinterpret_cast<const double*>(
                        sB(cur) + (wn * WN + j * 16 + li) * LDK + lg * (BK / 4) + s);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j],
                                                                         0, 0, 0);
                // keep the next step's fragment reads from being hoisted (their
                // registers would push the accumulators out of place)
                __builtin_amdgcn_sched_barrier(0);
            }
        } else if constexpr (sizeof(T) == 2) {
            // BF16: one 16-byte fragment per tile and step
#pragma unroll
            for (int s = 0; s < NSTEP; ++s) {
                uint4 fa[TM], fb[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    fa[i] = *reinterpret_cast<const uint4*>(
                        sA(cur) + (wm * WM + i * 16 + li) * LDK + lg * (BK / 4) + s * 8);
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    fb[j] = *reinterpret_cast<const uint4*>(
                        sB(cur) + (wn * WN + j * 16 + li) * LDK + lg * (BK / 4) + s * 8);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf8v, fa[i]), __builtin_bit_cast(bf8v, fb[j]),
                            acc[i][j], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            uint4 fa[TM][2], fb[TN][2];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const T* p = sA(cur) + (wm * WM + i * 16 + li) * LDK + lg * (BK / 4);
                fa[i][0] = reinterpret_cast<const uint4*>(p)[0];
                fa[i][1] = reinterpret_cast<const uint4*>(p)[1];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const T* p = sB(cur) + (wn * WN + j * 16 + li) * LDK + lg * (BK / 4);
                fb[j][0] = reinterpret_cast<const uint4*>(p)[0];
                fb[j][1] = reinterpret_cast<const uint4*>(p)[1];
            }
#pragma unroll
            for (int s = 0; s < NSTEP; ++s)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[i][j] = MT::step(fa[i], fb[j], s, acc[i][j]);
        }
    };

    // k-tiles that need no bounds checks: every full tile when both operands
    // are vector-aligned; the ragged k tail (and unaligned operands) are guarded
    const long long nk = (g.K + BK - 1) / BK;
    const long long nfast = (g.vecA && g.vecB) ? g.K / BK : 0;
    if (nk > 0) {
        if (nfast > 0) {
            load_fast(A, g.lda, TrA{}, m0, g.M, BM, ra, CA, 0);
            load_fast(B, g.ldb, TrB{}, n0, g.N, BN, rb, CB, 0);
        } else {
            load_safe(A, g.lda, TrA{}, m0, g.M, BM, ra, CA, 0);
            load_safe(B, g.ldb, TrB{}, n0, g.N, BN, rb, CB, 0);
        }
        store(sA(0), TrA{}, BM, ra, CA);
        store(sB(0), TrB{}, BN, rb, CB);
        __syncthreads();
        long long kt = 0;
        // the next tile is a fast one
        for (; kt + 1 < nfast; ++kt) {
            const int cur = kt & 1;
            load_fast(A, g.lda, TrA{}, m0, g.M, BM, ra, CA, (kt + 1) * BK);
            load_fast(B, g.ldb, TrB{}, n0, g.N, BN, rb, CB, (kt + 1) * BK);
            compute(cur);
            store(sA(cur ^ 1), TrA{}, BM, ra, CA);
            store(sB(cur ^ 1), TrB{}, BN, rb, CB);
            __syncthreads();
        }
        // the next tile needs bounds checks
        for (; kt + 1 < nk; ++kt) {
            const int cur = kt & 1;
            load_safe(A, g.lda, TrA{}, m0, g.M, BM, ra, CA, (kt + 1) * BK);
            load_safe(B, g.ldb, TrB{}, n0, g.N, BN, rb, CB, (kt + 1) * BK);
            compute(cur);
            store(sA(cur ^ 1), TrA{}, BM, ra, CA);
            store(sB(cur ^ 1), TrB{}, BN, rb, CB);
            __syncthreads();
        }
        compute(kt & 1);
    }

    // ---- epilogue: staged through the operand tiles' LDS ----------------
    constexpr int NW = WGM * WGN;
    constexpr int SMEM_BYTES = 2 * (BM + BN) * LDK * (int)sizeof(T);
    constexpr int PAD = 16 / (int)sizeof(acc_t);
    constexpr int NPASS = (NW * WM * (WN + PAD) * (int)sizeof(acc_t) <= SMEM_BYTES)         ? 1
                          : (NW * WM * (WN / 2 + PAD) * (int)sizeof(acc_t) <= SMEM_BYTES) ? 2
                                                                                            : 4;
    static_assert(NW * WM * (WN / NPASS + PAD) * (int)sizeof(acc_t) <= SMEM_BYTES,
                  "epilogue staging");
    acc_t* stage = reinterpret_cast<acc_t*>(smem) + wave * (WM * (WN / NPASS + PAD));
    store_tile<T, TO, WM, WN, NPASS>(acc, stage, C, g, m0 + wm * WM, n0 + wn * WN, lane, alpha,
                                     beta);
}

// BF16 NT product (A [M][K], B [N][K], both k-fastest) on a 256x256 tile of
// 8 waves (4 x 2, a 64x128 block each) whose operand tiles go from global
// memory straight into LDS with 16-byte LDS-DMA loads (global_load_lds): no
// staging registers and no LDS store instructions, so the loads of the next
// k-tile are issued before the products of the current one and have a whole
// k-step to arrive.  Each operand and stage has an LDS array of its own: the
// compiler then knows that the outstanding loads write the other stage, and
// the fragment reads of this one need not wait for them.
//
// LDS layout of an operand tile: row r (0..255) of 64 k-values in 128 bytes,
// its 16-byte chunk c (k = 8c .. 8c+7) at position c ^ (r mod 8).  One DMA
// instruction of a wave fills 1 KB (8 rows) with lane l writing position
// l mod 8 of row l / 8, so each lane loads the chunk that the XOR puts there.
// The fragment reads of 8 consecutive rows at one chunk hit 8 distinct 16-byte
// bank groups.  Full k-tiles need every row in bounds: rows past the operand's
// extent are clamped to its last row (they only feed discarded outputs); the
// ragged last k-tile is loaded through registers with zero fill.
template <typename TO, int KIND>
__global__ void __launch_bounds__(512)
k_gemm_lds(const bf16_t* __restrict__ A, const bf16_t* __restrict__ B, TO* __restrict__ C,
           GemmShape g, float alpha, float beta) {
    using MT = Mfma<bf16_t>;
    using accv = typename MT::accv;
    constexpr int BM = 256, BN = 256, BK = 64, WGN = 2, NW = 8;
    constexpr int WM = 64, WN = 128, TM = WM / 16, TN = WN / 16;
    constexpr int ROWB = BK * 2;                      // bytes per LDS row
    constexpr int NPASS = 2, LDC = WN / NPASS + 4;    // epilogue: FP32 rows of 68
    constexpr int STAGE = WM * LDC * 4;               // epilogue bytes per wave
    constexpr int BUF = (BM * ROWB > 2 * STAGE) ? BM * ROWB : 2 * STAGE;
    constexpr int NBLK = BM * ROWB / 1024 / NW;       // 1 KB DMA blocks per wave and tile
    static_assert(BM == BN && BM * ROWB == 32768 && NBLK * NW * 1024 == 32768,
                  "operand tile layout");
    __shared__ __attribute__((aligned(1024))) char la0[BUF], la1[BUF], lb0[BUF], lb1[BUF];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WGN, wn = wave % WGN;
    const int li = lane & 15, lg = lane >> 4;

    long long m0, n0;
    tile_origin<BM, BN>(g, m0, n0);
    {
        const BatchOff o = batch_offsets(g);
        A += o.a;
        B += o.b;
        C += o.c;
    }

    // this lane's NBLK rows of each operand tile (1 KB blocks wave, wave + NW,
    // ...) and the k-chunk it loads into each
    const int rl = lane >> 3;
    const int kc = (lane & 7) ^ rl;
    const bf16_t* pa[NBLK];
    const bf16_t* pb[NBLK];
#pragma unroll
    for (int j = 0; j < NBLK; ++j) {
        const int r = 8 * (wave + NW * j) + rl;
        const long long ra = m0 + r < g.M ? m0 + r : g.M - 1;
        const long long rb = n0 + r < g.N ? n0 + r : g.N - 1;
        pa[j] = A + ra * g.lda + kc * 8;
        pb[j] = B + rb * g.ldb + kc * 8;
    }
    typedef __attribute__((address_space(1))) void gvoid;
    typedef __attribute__((address_space(3))) void lvoid;
    // a full k-tile (k0 + BK <= K) by DMA
    auto dma = [&](char* sa, char* sb, long long k0) {
#pragma unroll
        for (int j = 0; j < NBLK; ++j) {
            __builtin_amdgcn_global_load_lds((gvoid*)(pa[j] + k0),
                                             (lvoid*)(sa + (wave + NW * j) * 1024), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((gvoid*)(pb[j] + k0),
                                             (lvoid*)(sb + (wave + NW * j) * 1024), 16, 0, 0);
        }
    };
    // the ragged last k-tile through registers: chunks inside K are one
    // 16-byte load, chunks past K (or of rows past the operand) are zero, and
    // a chunk that K cuts (K not a multiple of 8) is read element by element
    auto tail = [&](char* sa, char* sb, long long k0) {
        const long long k = k0 + kc * 8;
#pragma unroll
        for (int j = 0; j < NBLK; ++j) {
            const int r = 8 * (wave + NW * j) + rl;
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                const bf16_t* p = (o == 0 ? pa[j] : pb[j]) + k0;
                const bool row_ok = o == 0 ? m0 + r < g.M : n0 + r < g.N;
                uint4 v = {0u, 0u, 0u, 0u};
                if (row_ok && k + 8 <= g.K) {
                    v = *reinterpret_cast<const uint4*>(p);
                } else if (row_ok && k < g.K) {
                    bf16_t e8[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) e8[e] = k + e < g.K ? p[e] : bf16_t(0);
                    v = __builtin_bit_cast(uint4, e8);
                }
                *reinterpret_cast<uint4*>((o == 0 ? sa : sb) + (wave + NW * j) * 1024 + lane * 16) =
                    v;
            }
        }
    };

    accv acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = accv{};

    // one k-tile: two steps of k = 32; lane (li, lg) takes chunk 2 lg + s of
    // its rows (rows li mod 8 = li & 7 in every 16-row block)
    auto compute = [&](const char* sa, const char* sb) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int u = ((2 * lg + s) ^ (li & 7)) * 16;
            uint4 fa[TM], fb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                fa[i] = *reinterpret_cast<const uint4*>(sa + (wm * WM + i * 16 + li) * ROWB + u);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                fb[j] = *reinterpret_cast<const uint4*>(sb + (wn * WN + j * 16 + li) * ROWB + u);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf8v, fa[i]), __builtin_bit_cast(bf8v, fb[j]),
                        acc[i][j], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // full k-tiles: the stages alternate statically (two k-tiles per trip),
    // so every LDS access names its array
    const long long nfull = g.K / BK;
    if (nfull > 0) {
        dma(la0, lb0, 0);
        __syncthreads();
        for (long long kt = 0;;) {
            if (kt + 1 < nfull) dma(la1, lb1, (kt + 1) * BK);
            compute(la0, lb0);
            __syncthreads();
            if (++kt == nfull) break;
            if (kt + 1 < nfull) dma(la0, lb0, (kt + 1) * BK);
            compute(la1, lb1);
            __syncthreads();
            if (++kt == nfull) break;
        }
    }
    // the ragged last k-tile (every stage is free after the barrier above)
    if (nfull * BK < g.K) {
        tail(la0, lb0, nfull * BK);
        __syncthreads();
        compute(la0, lb0);
    }

    // epilogue: waves 2w and 2w+1 stage their blocks in array w
    char* base = wave < 2 ? la0 : wave < 4 ? la1 : wave < 6 ? lb0 : lb1;
    float* stage = reinterpret_cast<float*>(base + (wave & 1) * STAGE);
    store_tile<bf16_t, TO, WM, WN, NPASS>(acc, stage, C, g, m0 + wm * WM, n0 + wn * WN, lane,
                                          alpha, beta);
}

static bool aligned16(const void* p) {
    return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

template <typename TI, typename T, typename TO, int BM, int BN, int WGM, int WGN, int KIND>
static void launch_tiles(hipStream_t st, bool ta, bool tb, const TI* A, const TI* B, TO* C,
                         const GemmShape& g, long long batch, typename Mfma<T>::acc_t alpha,
                         typename Mfma<T>::acc_t beta) {
    const long long ntm = (g.M + BM - 1) / BM, ntn = (g.N + BN - 1) / BN;
    ADC_REQUIRE(ntm * ntn * 64 * WGM * WGN < (1LL << 32), "gemm: grid too large");
    constexpr int NT = 64 * WGM * WGN;
    // the batch index runs over grid z (at most 65535 per launch)
    for (long long z0 = 0; z0 < batch; z0 += 65535) {
        const long long nz = std::min<long long>(65535, batch - z0);
        GemmShape gz = g;
        gz.z0 = z0;
        dim3 grid((unsigned)(ntm * ntn), 1, (unsigned)nz);
        if (KIND != 0 || (!ta && tb))
            hipLaunchKernelGGL((k_gemm<TI, T, TO, BM, BN, WGM, WGN, false, true, KIND>), grid,
                               dim3(NT), 0, st, A, B, C, gz, alpha, beta);
        else if (!ta && !tb)
            hipLaunchKernelGGL((k_gemm<TI, T, TO, BM, BN, WGM, WGN, false, false, 0>), grid,
                               dim3(NT), 0, st, A, B, C, gz, alpha, beta);
        else if (ta && !tb)
            hipLaunchKernelGGL((k_gemm<TI, T, TO, BM, BN, WGM, WGN, true, false, 0>), grid,
                               dim3(NT), 0, st, A, B, C, gz, alpha, beta);
        else
            hipLaunchKernelGGL((k_gemm<TI, T, TO, BM, BN, WGM, WGN, true, true, 0>), grid,
                               dim3(NT), 0, st, A, B, C, gz, alpha, beta);
        ADC_HIP(hipGetLastError());
    }
}

// Launch of the LDS-DMA BF16 tile (configuration 8) over the batch.
template <typename TO, int KIND>
static void launch_lds_tiles(hipStream_t st, const bf16_t* A, const bf16_t* B, TO* C,
                             const GemmShape& g, long long batch, float alpha, float beta) {
    const long long ntm = (g.M + 255) / 256, ntn = (g.N + 255) / 256;
    ADC_REQUIRE(ntm * ntn * 512 < (1LL << 32), "gemm: grid too large");
    for (long long z0 = 0; z0 < batch; z0 += 65535) {
        const long long nz = std::min<long long>(65535, batch - z0);
        GemmShape gz = g;
        gz.z0 = z0;
        hipLaunchKernelGGL((k_gemm_lds<TO, KIND>), dim3((unsigned)(ntm * ntn), 1, (unsigned)nz),
                           dim3(512), 0, st, A, B, C, gz, alpha, beta);
        ADC_HIP(hipGetLastError());
    }
}

// Tile configurations: (BM, BN, waves in M, waves in N).
//   0: 64x64 (4x1)    1: 128x128 (2x2)   2: 128x128 (4x2)   3: 128x64 (2x2)
//   4: 256x128 (2x2)  5: 256x256 (2x2)   6: 256x128 (4x2)   7: 256x256 (4x2)
//   8: 256x256 (4x2), BF16 NT with operands loaded straight into LDS
//      (k_gemm_lds; other products given 8 run as 7)
// The 8-wave 256x256 tile gives each wave a 64x128 block: half the LDS reads
// per multiply of the 64x64 blocks, which is what limits BF16. For FP64
// the 4-wave 64x64 tile (four workgroups per CU) beats larger tiles on
// products with few rows and a long summed index, such as the 320-row
// particle-particle contraction: occupancy hides more latency than the larger
// tiles save in operand reads.

// configurations compiled for each compute type (the rest fall back to 0)
template <typename T> static bool cfg_available(int cfg);
template <> inline bool cfg_available<double>(int cfg) {
    return cfg == 0 || cfg == 2 || cfg == 3;
}
template <> inline bool cfg_available<float>(int cfg) { return cfg == 0 || cfg == 1 || cfg == 2; }
template <> inline bool cfg_available<bf16_t>(int cfg) {
    return cfg == 0 || cfg == 1 || cfg == 6 || cfg == 7 || cfg == 8;
}

// untuned choice: the large tile when both sides fill it and the grid gives
// the chip at least one (256x256) or two (128x128) rounds of workgroups, else
// 64x64
template <typename T>
static int choose_cfg(long long M, long long N, long long batch) {
    auto wgs = [&](int bm, int bn) { return ((M + bm - 1) / bm) * ((N + bn - 1) / bn) * batch; };
    const bool big = M >= 256 && N >= 256 && wgs(128, 128) >= 512;
    if (sizeof(T) == 8) return big ? 2 : 0;
    if (sizeof(T) == 2 && M >= 512 && N >= 512 && wgs(256, 256) >= 256) return 7;
    return big ? 1 : 0;
}

extern int g_force_cfg;   // tuning override (all types), -1: automatic

template <typename TI, typename T, typename TO>
void mfma_gemm(hipStream_t st, bool ta, bool tb, long long M, long long N, long long K,
               typename AccOf<T>::type alpha, const TI* A, long long lda, long long sA, const TI* B,
               long long ldb, long long sB, typename AccOf<T>::type beta, TO* C, GemmOut out,
               long long batch, int kind, int cfg_req, GemmInner inner) {
    if (M <= 0 || N <= 0 || batch <= 0 || inner.n <= 0) return;
    ADC_REQUIRE(inner.n == 1 || batch * inner.n <= 65535, "gemm: two-level batch too large");
    ADC_REQUIRE(kind == 0 || (!ta && tb), "gemm: tagged kernels are NT only");
    ADC_REQUIRE(K >= 0 && lda >= (ta ? M : K) && ldb >= (tb ? K : N), "gemm: leading dimension");
    ADC_REQUIRE(A && B && C, "gemm: null operand");
    GemmShape g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = lda;
    g.ldb = ldb;
    g.sA = sA;
    g.sB = sB;
    g.sC = out.sC;
    g.rsplit = out.rsplit > 0 ? out.rsplit : M;
    g.rs1 = out.rs1;
    g.rs2 = out.rs2;
    g.csplit = out.csplit > 0 ? out.csplit : N;
    g.cs1 = out.cs1;
    g.cs2 = out.cs2;
    g.n2 = inner.n;
    g.sA2 = inner.sA;
    g.sB2 = inner.sB;
    g.sC2 = inner.sC;
    g.z0 = 0;
    // the two levels run as one flat batch over grid z
    batch *= inner.n;
    // 16-byte loads: every offset a multiple of VWI storage elements; a
    // [k][row] operand also needs whole VW-element chunks per k-row (the
    // clamp of rows past the extent relies on it)
    constexpr int VW = 16 / sizeof(T), VWI = 16 / sizeof(TI);
    const bool rowsA = ta, rowsB = !tb;     // [k][row] layouts
    g.vecA = aligned16(A) && (lda % (rowsA ? VW : VWI) == 0) && (batch == 1 || sA % VWI == 0) &&
             inner.sA % VWI == 0;
    g.vecB = aligned16(B) && (ldb % (rowsB ? VW : VWI) == 0) && (batch == 1 || sB % VWI == 0) &&
             inner.sB % VWI == 0;
    if (K <= 0) {
        // nothing to accumulate: C = beta C through the same epilogue
        g.K = 0;
    }
    // tile choice: 128x128 for large problems, 64x64 when the grid would be small
    int cfg = g_force_cfg >= 0 ? g_force_cfg : cfg_req >= 0 ? cfg_req : choose_cfg<T>(M, N, batch);
    if (!cfg_available<T>(cfg)) cfg = 0;
#define ADC_CFG(ID, BM, BN, WM, WN)                                                             \
    case ID:                                                                                    \
        if (kind == 1)                                                                          \
            launch_tiles<TI, T, TO, BM, BN, WM, WN, 1>(st, ta, tb, A, B, C, g, batch, alpha, beta); \
        else if (kind == 2)                                                                     \
            launch_tiles<TI, T, TO, BM, BN, WM, WN, 2>(st, ta, tb, A, B, C, g, batch, alpha, beta); \
        else                                                                                    \
            launch_tiles<TI, T, TO, BM, BN, WM, WN, 0>(st, ta, tb, A, B, C, g, batch, alpha, beta); \
        break;
    if constexpr (sizeof(T) == 8) {
        switch (cfg) {
            ADC_CFG(2, 128, 128, 4, 2)
            ADC_CFG(3, 128, 64, 2, 2)
            default: ADC_CFG(0, 64, 64, 4, 1)
        }
    } else if constexpr (sizeof(T) == 4) {
        switch (cfg) {
            ADC_CFG(1, 128, 128, 2, 2)
            ADC_CFG(2, 128, 128, 4, 2)
            default: ADC_CFG(0, 64, 64, 4, 1)
        }
    } else {
        // configuration 8 needs BF16 storage, the NT form and 16-byte aligned rows
        if (cfg == 8) {
            if constexpr (std::is_same<TI, bf16_t>::value) {
                if (!ta && tb && g.vecA && g.vecB) {
                    if (kind == 1)
                        launch_lds_tiles<TO, 1>(st, A, B, C, g, batch, alpha, beta);
                    else if (kind == 2)
                        launch_lds_tiles<TO, 2>(st, A, B, C, g, batch, alpha, beta);
                    else
                        launch_lds_tiles<TO, 0>(st, A, B, C, g, batch, alpha, beta);
                    return;
                }
            }
            cfg = 7;
        }
        switch (cfg) {
            ADC_CFG(1, 128, 128, 2, 2)
            ADC_CFG(6, 256, 128, 4, 2)
            ADC_CFG(7, 256, 256, 4, 2)
            default: ADC_CFG(0, 64, 64, 4, 1)
        }
    }
#undef ADC_CFG
}

}  // namespace adc
