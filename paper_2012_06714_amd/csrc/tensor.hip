// Tensor helpers: permutation kernel, row-major GEMM on the matrix-core kernel and
// an einsum-style binary contraction that maps onto (strided, batched) GEMM.
#include "adc_internal.hpp"
#include "mfma_gemm.hpp"

#include <algorithm>
#include <cstring>
#include <map>

namespace adc {

long long Ext::of(char c) const {
    if (c >= 'i' && c <= 'o') return O;
    if (c >= 'a' && c <= 'h') return V;
    if (c == 'Q') return Q;
    if (c == 'z') return Z;
    auto it = extra.find(c);
    if (it == extra.end()) throw Error(ADC_E_ARG, std::string("no extent for index ") + c);
    return it->second;
}

// ---------------------------------------------------------------------------
// permutation
// ---------------------------------------------------------------------------
struct PermArgs {
    int nd;
    long long dim[8];      // output extents (output order)
    long long istr[8];     // input stride of each output axis
};

template <typename T>
__global__ void k_permute(const T* __restrict__ in, T* __restrict__ out, PermArgs a, long long total,
                          T alpha, T beta) {
    long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long step = (long long)gridDim.x * blockDim.x;
    for (; o < total; o += step) {
        long long r = o, off = 0;
        for (int k = a.nd - 1; k >= 0; --k) {
            long long q = r / a.dim[k];
            off += (r - q * a.dim[k]) * a.istr[k];
            r = q;
        }
        T v = alpha * in[off];
        out[o] = (beta == T(0)) ? v : beta * out[o] + v;
    }
}

static unsigned grid_for(long long n, int bs = 256) {
    long long g = (n + bs - 1) / bs;
    if (g > 65536LL * 8) g = 65536LL * 8;
    if (g < 1) g = 1;
    return (unsigned)g;
}

template <typename T>
void permute(Engine& E, T alpha, const char* si, const T* in, T beta, const char* so, T* out) {
    int nd = (int)strlen(so);
    ADC_REQUIRE(nd == (int)strlen(si) && nd <= 8, "permute: rank mismatch");
    long long istr_in[8];
    long long s = 1;
    for (int k = nd - 1; k >= 0; --k) {
        istr_in[k] = s;
        s *= E.ext.of(si[k]);
    }
    PermArgs a;
    a.nd = nd;
    long long total = 1;
    for (int k = 0; k < nd; ++k) {
        const char* p = strchr(si, so[k]);
        ADC_REQUIRE(p, "permute: letter missing");
        a.dim[k] = E.ext.of(so[k]);
        a.istr[k] = istr_in[p - si];
        total *= a.dim[k];
    }
    if (total == 0) return;
    hipLaunchKernelGGL(k_permute<T>, dim3(grid_for(total)), dim3(256), 0, E.stream, in, out, a,
                       total, alpha, beta);
    ADC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// GEMM (row-major view over column-major rocBLAS)
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// GEMM autotuner
// ---------------------------------------------------------------------------
template <typename TI, typename T, typename TO>
void gemm_run(Engine& E, bool ta, bool tb, long long M, long long N, long long K,
              typename AccOf<T>::type alpha, const TI* A, long long lda, long long sA,
              const TI* B, long long ldb, long long sB, typename AccOf<T>::type beta, TO* C,
              GemmOut out, long long batch, int kind, GemmInner inner) {
    using Acc = typename AccOf<T>::type;
    if (M <= 0 || N <= 0 || batch <= 0 || inner.n <= 0) return;
    // shapes are tuned per class (each extent rounded up to a power of two):
    // loops whose products differ only a little in one extent (the particle-
    // particle groups) reuse one trial instead of timing every shape
    auto cls = [](long long x) {
        long long p = 1;
        while (p < x) p <<= 1;
        return p;
    };
    const std::array<long long, 12> key{(long long)sizeof(TI), (long long)sizeof(T),
                                        (long long)sizeof(TO), ta, tb, cls(M), cls(N), cls(K),
                                        cls(batch * inner.n), kind, out.rsplit > 0,
                                        out.csplit > 0};
    if (E.force_cfg >= 0) {   // a forced tile (configurations not compiled for T run as 0)
        mfma_gemm<TI, T, TO>(E.stream, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C,
                             out, batch, kind, E.force_cfg, inner);
        return;
    }
    auto it = E.tuned.find(key);
    if (it != E.tuned.end()) {
        mfma_gemm<TI, T, TO>(E.stream, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C,
                             out, batch, kind, it->second, inner);
        return;
    }
    const double flops = 2.0 * M * N * K * batch * inner.n;
    const size_t cbytes = sizeof(TO) * (size_t)M * N * batch * inner.n;
    // trials of a two-level batch would need a scratch copy of its whole
    // strided output: those shapes take the heuristic choice
    if (!E.autotune || flops < 2e8 || (beta != Acc(0) && (cbytes > (size_t(512) << 20) || inner.n > 1))) {
        mfma_gemm<TI, T, TO>(E.stream, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C,
                             out, batch, kind, -1, inner);
        return;
    }
    // trials: in place when the product overwrites C, else on a scratch output
    TO* Ct = C;
    GemmOut ot = out;
    Acc bt = beta;
    GemmInner it2 = inner;
    if (beta != Acc(0)) {
        Ct = (TO*)E.scratch.get(28, cbytes);
        ot = GemmOut::rowmajor(N, M * N);
        bt = Acc(0);
    }
    if (!E.tev[0]) {
        ADC_HIP(hipEventCreate(&E.tev[0]));
        ADC_HIP(hipEventCreate(&E.tev[1]));
    }
    int ids[8];
    const int n = gemm_candidates<T>(ids);
    float ms_of[8];
    auto trial = [&](int k) {
        ADC_HIP(hipEventRecord(E.tev[0], E.stream));
        mfma_gemm<TI, T, TO>(E.stream, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, bt, Ct, ot,
                             batch, kind, ids[k], it2);
        ADC_HIP(hipEventRecord(E.tev[1], E.stream));
        ADC_HIP(hipEventSynchronize(E.tev[1]));
        float ms = 0.f;
        ADC_HIP(hipEventElapsedTime(&ms, E.tev[0], E.tev[1]));
        return ms;
    };
    // configuration 8 (LDS-DMA loads) only exists for BF16 storage in the NT
    // form; elsewhere it would run as 7 and need no trial of its own
    const bool lds_ok = std::is_same<TI, bf16_t>::value && !ta && tb;
    for (int k = 0; k < n; ++k) ms_of[k] = (ids[k] == 8 && !lds_ok) ? 3.0e38f : trial(k);
    // a close second (within 10 %) is timed again together with the leader,
    // runner-up first, and each keeps its faster time: one launch of a few
    // milliseconds is too noisy (clock changes between launches) to separate them
    int b1 = 0, b2 = -1;
    for (int k = 1; k < n; ++k)
        if (ms_of[k] < ms_of[b1]) b1 = k;
    for (int k = 0; k < n; ++k)
        if (k != b1 && (b2 < 0 || ms_of[k] < ms_of[b2])) b2 = k;
    if (b2 >= 0 && ms_of[b2] < 1.10f * ms_of[b1]) {
        ms_of[b2] = std::min(ms_of[b2], trial(b2));
        ms_of[b1] = std::min(ms_of[b1], trial(b1));
        if (ms_of[b2] < ms_of[b1]) b1 = b2;
    }
    const int bc = ids[b1];
    const float best = ms_of[b1];
    E.tuned[key] = bc;
    if (E.tune_log) {
        fprintf(stderr, "gemm tune: in %d B cmp %d B out %d B %c%c M %lld N %lld K %lld batch %lld "
                "kind %d -> config %d (%.3f ms, %.1f TFLOP/s); candidates",
                (int)sizeof(TI), (int)sizeof(T), (int)sizeof(TO), ta ? 'T' : 'N', tb ? 'T' : 'N',
                M, N, K, batch * inner.n, kind, bc, best, flops / (best * 1e-3) / 1e12);
        for (int k = 0; k < n; ++k) fprintf(stderr, " %d: %.3f ms", ids[k], ms_of[k]);
        fprintf(stderr, "\n");
    }
    if (Ct != C)
        mfma_gemm<TI, T, TO>(E.stream, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C,
                             out, batch, kind, bc, inner);
}

#define ADC_RUN_INST(TI, T, TO)                                                                  \
    template void gemm_run<TI, T, TO>(Engine&, bool, bool, long long, long long, long long,      \
                                      AccOf<T>::type, const TI*, long long, long long, const TI*, \
                                      long long, long long, AccOf<T>::type, TO*, GemmOut,         \
                                      long long, int, GemmInner);
ADC_RUN_INST(double, double, double)
ADC_RUN_INST(float, float, float)
ADC_RUN_INST(float, bf16_t, float)
ADC_RUN_INST(bf16_t, bf16_t, float)
ADC_RUN_INST(bf16_t, bf16_t, bf16_t)
ADC_RUN_INST(float, bf16_t, bf16_t)
ADC_RUN_INST(float, float, bf16_t)
#undef ADC_RUN_INST

// Skinny products with a long summed index (Davidson overlaps, gemv-like
// contractions, small batched products) would leave most of the chip idle:
// split K into chunks run as the inner level of a two-level batched GEMM
// into partial results [chunk][batch][M][N], then reduce them in a fixed order.
template <typename A>
__global__ void k_splitk_reduce(const A* __restrict__ part, int S, long long batch, long long M,
                                long long N, A* __restrict__ C, GemmOut o, A beta) {
    // block: 64 consecutive outputs (one per lane, coalesced) x G chunk groups
    // (blockDim.y); group g sums chunks g, g+G, ..., then group 0 adds the G
    // partial sums in order: a fixed summation order for every launch
    __shared__ A red[16][64];
    const long long MN = M * N, tot = batch * MN;
    const int lane = threadIdx.x, g = threadIdx.y, G = blockDim.y;
    const long long e = (long long)blockIdx.x * 64 + lane;
    A v = 0;
    if (e < tot)
        for (int s = g; s < S; s += G) v += part[(long long)s * tot + e];
    red[g][lane] = v;
    __syncthreads();
    if (g != 0 || e >= tot) return;
    A sum = 0;
    for (int k = 0; k < G; ++k) sum += red[k][lane];
    const long long rsplit = o.rsplit > 0 ? o.rsplit : M, csplit = o.csplit > 0 ? o.csplit : N;
    const long long b = e / MN, r = e - b * MN;
    const long long m = r / N, n = r - m * N;
    const long long m1 = m / rsplit, n1 = n / csplit;
    A* dst = C + b * o.sC + m1 * o.rs1 + (m - m1 * rsplit) * o.rs2 + n1 * o.cs1 +
             (n - n1 * csplit) * o.cs2;
    *dst = (beta == A(0)) ? sum : beta * *dst + sum;
}

// number of k-chunks for a product of `wgs` 64x64 workgroups: enough chunks
// to give the chip about 1024 workgroups, each chunk at least 512 long, the
// partial results at most 256 MiB
static long long splitk_chunks(long long M, long long N, long long K, long long batch, size_t acc) {
    const long long wgs = ((M + 63) / 64) * ((N + 63) / 64) * batch;
    if (wgs >= 256 || K < 1024) return 1;
    long long S = std::min<long long>((1024 + wgs - 1) / wgs, K / 512);
    S = std::min<long long>(S, 65535 / batch);
    const long long cap = (long long)((size_t(256) << 20) / (acc * (size_t)(M * N * batch)));
    S = std::min(S, cap);
    return std::max<long long>(S, 1);
}

// BF16 particle-particle contractions (kind 2): a few hundred 256x256
// workgroups over a summed index of V^2, one workgroup per CU, lose up to half
// the chip in their last round.  Split K when that raises the filled share of
// the rounds (the first s-1 chunks are one launch, the last another) by more
// than 5 points (each chunk at least 4096 long, the partial results at most
// 1 GiB, at most 8 chunks).
static long long splitk_rounds(long long M, long long N, long long K, long long batch, size_t acc) {
    const long long n = ((M + 255) / 256) * ((N + 255) / 256) * batch;
    // chunks 0 .. s-2 run as one launch and the last chunk as another
    auto rounds = [](long long w) { return (w + 255) / 256; };
    auto filled = [&](long long s) {
        const long long r = s == 1 ? rounds(n) : rounds(n * (s - 1)) + rounds(n);
        return (double)(n * s) / (256.0 * (double)r);
    };
    long long best = 1;
    double fb = filled(1);
    for (long long s = 2; s <= 8; ++s) {
        if (K / s < 4096 || s * batch > 65535) break;
        if ((size_t)s * (size_t)(M * N * batch) * acc > (size_t(1) << 30)) break;
        if (filled(s) > fb + 0.05) {
            best = s;
            fb = filled(s);
        }
    }
    return best;
}

// C (accumulator type) = alpha op(A) op(B) + beta C, row-major output with
// leading dimension ldc, through split-K when the grid would be small
template <typename TI, typename T>
static void gemm_any(Engine& E, bool ta, bool tb, long long M, long long N, long long K,
                     typename AccOf<T>::type alpha, const TI* A, long long lda, long long sA,
                     const TI* B, long long ldb, long long sB, typename AccOf<T>::type beta,
                     typename AccOf<T>::type* C, GemmOut out, long long batch, int kind) {
    using Acc = typename AccOf<T>::type;
    long long S = (sizeof(T) == 2 && kind == 2) ? splitk_rounds(M, N, K, batch, sizeof(Acc))
                                                : splitk_chunks(M, N, K, batch, sizeof(Acc));
    long long Kc = K;
    if (S >= 2) {
        Kc = (K + S - 1) / S;
        Kc = (Kc + 63) / 64 * 64;
        S = (K + Kc - 1) / Kc;
    }
    if (S >= 2 && (kind == 0 || (!ta && tb))) {
        const long long Klast = K - (S - 1) * Kc;
        const long long MNB = M * N * batch;
        Acc* part = (Acc*)E.scratch.get(31, sizeof(Acc) * S * MNB);
        // k offsets of one chunk in A and B
        const long long offA = ta ? Kc * lda : Kc, offB = tb ? Kc : Kc * ldb;
        GemmInner in;
        in.n = S - 1;
        in.sA = offA;
        in.sB = offB;
        in.sC = MNB;
        // chunks 0 .. S-2 (inner level) of every batch item (outer level)
        gemm_run<TI, T, Acc>(E, ta, tb, M, N, Kc, alpha, A, lda, sA, B, ldb, sB, Acc(0), part,
                             GemmOut::rowmajor(N, M * N), batch, kind, in);
        gemm_run<TI, T, Acc>(E, ta, tb, M, N, Klast, alpha, A + (S - 1) * offA, lda, sA,
                             B + (S - 1) * offB, ldb, sB, Acc(0), part + (S - 1) * MNB,
                             GemmOut::rowmajor(N, M * N), batch, kind);
        const long long nb = (MNB + 63) / 64;
        ADC_REQUIRE(nb < (1LL << 31), "split-K: too many outputs");
        const int G = (int)std::min<long long>(16, S);
        hipLaunchKernelGGL(k_splitk_reduce<Acc>, dim3((unsigned)nb), dim3(64, G), 0, E.stream,
                           part, (int)S, batch, M, N, C, out, beta);
        ADC_HIP(hipGetLastError());
        return;
    }
    gemm_run<TI, T, Acc>(E, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, out, batch,
                         kind);
}

template <typename TI, typename T>
void gemm_acc(Engine& E, bool ta, bool tb, long long M, long long N, long long K,
              typename AccOf<T>::type alpha, const TI* A, long long lda, const TI* B, long long ldb,
              typename AccOf<T>::type beta, typename AccOf<T>::type* C, GemmOut out, int kind) {
    gemm_any<TI, T>(E, ta, tb, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, out, 1, kind);
}
template void gemm_acc<double, double>(Engine&, bool, bool, long long, long long, long long, double,
                                       const double*, long long, const double*, long long, double,
                                       double*, GemmOut, int);
template void gemm_acc<bf16_t, bf16_t>(Engine&, bool, bool, long long, long long, long long, float,
                                       const bf16_t*, long long, const bf16_t*, long long, float,
                                       float*, GemmOut, int);
template void gemm_acc<float, float>(Engine&, bool, bool, long long, long long, long long, float,
                                     const float*, long long, const float*, long long, float,
                                     float*, GemmOut, int);

// compute type of an operand storage type: FP64 -> FP64, FP32 -> BF16 in the
// mixed mode (FP32 otherwise), BF16 -> BF16
template <typename TI> struct CompOf { using type = TI; };
template <> struct CompOf<float> { using type = float; };

template <typename TI, typename TO>
void gemm_map(Engine& E, bool ta, bool tb, long long M, long long N, long long K, double alpha,
              const TI* A, long long lda, const TI* B, long long ldb, double beta, TO* C,
              GemmOut out) {
    if (M <= 0 || N <= 0) return;
    E.gemm_flops += 2LL * M * N * K;
    auto run = [&](auto tag) {
        using T = decltype(tag);
        using Acc = typename AccOf<T>::type;
        if constexpr (std::is_same<TO, Acc>::value) {
            gemm_any<TI, T>(E, ta, tb, M, N, K, (Acc)alpha, A, lda, 0, B, ldb, 0, (Acc)beta, C, out,
                            1, 0);
            return;
        }
        gemm_run<TI, T, TO>(E, ta, tb, M, N, K, (Acc)alpha, A, lda, 0, B, ldb, 0, (Acc)beta, C,
                            out, 1);
    };
    if constexpr (std::is_same<TI, float>::value) {
        if (E.bf16)
            run(bf16_t());
        else
            run(float());
    } else {
        run(TI());
    }
}

template void gemm_map<double, double>(Engine&, bool, bool, long long, long long, long long, double,
                                       const double*, long long, const double*, long long, double,
                                       double*, GemmOut);
template void gemm_map<float, float>(Engine&, bool, bool, long long, long long, long long, double,
                                     const float*, long long, const float*, long long, double,
                                     float*, GemmOut);
template void gemm_map<float, bf16_t>(Engine&, bool, bool, long long, long long, long long, double,
                                      const float*, long long, const float*, long long, double,
                                      bf16_t*, GemmOut);
template void gemm_map<bf16_t, float>(Engine&, bool, bool, long long, long long, long long, double,
                                      const bf16_t*, long long, const bf16_t*, long long, double,
                                      float*, GemmOut);
template void gemm_map<bf16_t, bf16_t>(Engine&, bool, bool, long long, long long, long long, double,
                                       const bf16_t*, long long, const bf16_t*, long long, double,
                                       bf16_t*, GemmOut);

template <>
void gemm_rm<double>(Engine& E, bool ta, bool tb, long long M, long long N, long long K, double alpha,
                     const double* A, long long lda, long long sA, const double* B, long long ldb,
                     long long sB, double beta, double* C, long long ldc, long long sC,
                     long long batch) {
    if (M == 0 || N == 0 || batch == 0) return;
    E.gemm_flops += 2LL * M * N * K * batch;
    gemm_any<double, double>(E, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C,
                             GemmOut::rowmajor(ldc, sC), batch, 0);
}

template <>
void gemm_rm<float>(Engine& E, bool ta, bool tb, long long M, long long N, long long K, float alpha,
                    const float* A, long long lda, long long sA, const float* B, long long ldb,
                    long long sB, float beta, float* C, long long ldc, long long sC,
                    long long batch) {
    if (M == 0 || N == 0 || batch == 0) return;
    E.gemm_flops += 2LL * M * N * K * batch;
    if (E.bf16)
        gemm_any<float, bf16_t>(E, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C,
                                GemmOut::rowmajor(ldc, sC), batch, 0);
    else
        gemm_any<float, float>(E, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C,
                               GemmOut::rowmajor(ldc, sC), batch, 0);
}

// ---------------------------------------------------------------------------
// einsum-style binary contraction
// ---------------------------------------------------------------------------
static bool has(const std::string& s, char c) { return s.find(c) != std::string::npos; }

template <typename T>
void ctr(Engine& E, T alpha, const char* sa_, const T* A, const char* sb_, const T* B, T beta,
         const char* sc_, T* C) {
    std::string sa(sa_), sb(sb_), sc(sc_);
    for (char c : sa) ADC_REQUIRE(has(sb, c) || has(sc, c), "ctr: index summed in one operand");
    for (char c : sb) ADC_REQUIRE(has(sa, c) || has(sc, c), "ctr: index summed in one operand");
    for (char c : sc) ADC_REQUIRE(has(sa, c) || has(sb, c), "ctr: output index missing");
    std::string batch, bcastA, bcastB, contr, fa, fb;
    for (char c : sc)
        if (has(sa, c) && has(sb, c)) batch += c;
    for (char c : sa)
        if (has(sb, c) && !has(sc, c)) contr += c;
    // free indices keep their order in the operand they come from
    for (char c : sa)
        if (has(sc, c) && !has(sb, c)) fa += c;
    for (char c : sb)
        if (has(sc, c) && !has(sa, c)) fb += c;
    // broadcast batching: leading free letters of an operand that also lead the
    // output may be looped over as a batch with zero stride in the other operand.
    // That is worth it only when it spares a permutation of that operand: else
    // the letters stay in the GEMM's M (or N), which gives larger tiles and
    // reads the other operand once per tile row instead of once per batch item.
    auto prefix_len = [](const std::string& x, const std::string& y) {
        size_t n = 0;
        while (n < x.size() && n < y.size() && x[n] == y[n]) ++n;
        return n;
    };
    auto usable = [&](const std::string& op, const std::string& lead, const std::string& f,
                      const std::string& k) { return op == lead + f + k || op == lead + k + f; };
    if (batch.empty()) {
        size_t nb = prefix_len(sb, sc);
        size_t k = 0;
        while (k < nb && has(fb, sb[k])) ++k;    // only letters that are free in B
        if (k > 0 && k < fb.size() && usable(sb, sb.substr(0, k), fb.substr(k), contr) &&
            !usable(sb, "", fb, contr)) {
            bcastB = sb.substr(0, k);
            fb = fb.substr(k);
        } else {
            size_t na = prefix_len(sa, sc);
            k = 0;
            while (k < na && has(fa, sa[k])) ++k;
            if (k > 0 && k < fa.size() && usable(sa, sa.substr(0, k), fa.substr(k), contr) &&
                !usable(sa, "", fa, contr)) {
                bcastA = sa.substr(0, k);
                fa = fa.substr(k);
            }
        }
    }
    auto ext = [&](const std::string& s) {
        long long n = 1;
        for (char c : s) n *= E.ext.of(c);
        return n;
    };
    const std::string lead = batch + bcastA + bcastB;
    long long nbatch = ext(lead);
    long long M = ext(fa), N = ext(fb), K = ext(contr);
    if (nbatch == 0 || M == 0 || N == 0) return;

    struct Log {
        Engine& e;
        hipEvent_t a = nullptr, b = nullptr;
        std::string text;
        double flops = 0;
        explicit Log(Engine& en) : e(en) {
            if (!e.ctr_log) return;
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            ADC_HIP(hipStreamIsCapturing(e.stream, &cs));
            if (cs != hipStreamCaptureStatusNone) return;    // no timing inside a capture
            ADC_HIP(hipEventCreate(&a));
            ADC_HIP(hipEventCreate(&b));
        }
        void start() { if (a) ADC_HIP(hipEventRecord(a, e.stream)); }
        ~Log() {
            if (!a) return;
            float ms = 0.f;
            if (hipEventRecord(b, e.stream) == hipSuccess && hipEventSynchronize(b) == hipSuccess)
                (void)hipEventElapsedTime(&ms, a, b);
            fprintf(stderr, "ctr %s: %.3f ms %.1f TFLOP/s\n", text.c_str(), ms,
                    flops / (ms * 1e-3 + 1e-30) / 1e12);
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } log(E);
    if (log.a) {
        char buf[512];
        snprintf(buf, sizeof buf, "%s,%s->%s M %lld N %lld K %lld batch %lld [%s|%s|%s] %c%c%s",
                 sa_, sb_, sc_, M, N, K, nbatch, batch.c_str(), bcastA.c_str(), bcastB.c_str(),
                 (sa == batch + bcastA + fa + contr) ? 'N' : (sa == batch + bcastA + contr + fa) ? 'T' : 'P',
                 (sb == batch + bcastB + contr + fb) ? 'N' : (sb == batch + bcastB + fb + contr) ? 'T' : 'P',
                 (sc == batch + bcastA + bcastB + fa + fb) ? "" :
                 (sc == batch + bcastA + bcastB + fb + fa) ? " Ct" : " Cp");
        log.text = buf;
        log.flops = 2.0 * M * N * K * nbatch;
        log.start();
    }
    // operand A: [lead'][fa][contr] or [lead'][contr][fa]; lead' = batch+bcastA
    const std::string leadA = batch + bcastA;
    bool ta = false;
    const T* Ause = A;
    if (sa == leadA + fa + contr) {
        ta = false;
    } else if (sa == leadA + contr + fa) {
        ta = true;
    } else {
        T* tmp = (T*)E.scratch.get(0, sizeof(T) * ext(sa));
        permute<T>(E, T(1), sa.c_str(), A, T(0), (leadA + fa + contr).c_str(), tmp);
        Ause = tmp;
        ta = false;
    }
    // operand B: [lead''][contr][fb] or [lead''][fb][contr]; contr order as in A
    const std::string leadB = batch + bcastB;
    bool tb = false;
    const T* Buse = B;
    if (sb == leadB + contr + fb) {
        tb = false;
    } else if (sb == leadB + fb + contr) {
        tb = true;
    } else {
        T* tmp = (T*)E.scratch.get(1, sizeof(T) * ext(sb));
        permute<T>(E, T(1), sb.c_str(), B, T(0), (leadB + contr + fb).c_str(), tmp);
        Buse = tmp;
        tb = false;
    }
    long long lda = ta ? M : K, ldb = tb ? K : N;
    long long sA = (long long)M * K, sB = (long long)K * N, sC = (long long)M * N;
    // result layout [batch][bcastA][bcastB][fa][fb]
    const std::string natural = batch + bcastA + bcastB + fa + fb;
    const std::string naturalT = batch + bcastA + bcastB + fb + fa;
    T* Cout = C;
    bool direct = (sc == natural), directT = (sc == naturalT);
    T beta_g = beta;
    if (!direct && !directT) {
        Cout = (T*)E.scratch.get(2, sizeof(T) * nbatch * M * N);
        beta_g = T(0);
    }
    // batch loops: batch letters stride through both operands; broadcast letters only one
    long long nb0 = ext(batch), nbA = ext(bcastA), nbB = ext(bcastB);
    for (long long b0 = 0; b0 < nb0; ++b0) {
        const T* Ab = Ause + b0 * nbA * sA;
        const T* Bb = Buse + b0 * nbB * sB;
        T* Cb = Cout + b0 * nbA * nbB * sC;
        // at most one of nbA, nbB exceeds 1: loop it as the GEMM batch
        long long nbat = nbA > 1 ? nbA : nbB;
        long long bsA = nbA > 1 ? sA : 0, bsB = nbA > 1 ? 0 : sB;
        if (directT) {
            // C^T = B^T A^T
            gemm_rm<T>(E, !tb, !ta, N, M, K, alpha, Bb, ldb, bsB, Ab, lda, bsA, beta_g, Cb, M, sC,
                       nbat);
        } else {
            gemm_rm<T>(E, ta, tb, M, N, K, alpha, Ab, lda, bsA, Bb, ldb, bsB, beta_g, Cb, N, sC,
                       nbat);
        }
    }
    if (!direct && !directT) {
        permute<T>(E, T(1), natural.c_str(), Cout, beta, sc.c_str(), C);
    }
}

// ---------------------------------------------------------------------------
// elementwise
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, T v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
template <typename T>
__global__ void k_axpy(T a, const T* x, T* y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}
__global__ void k_d2f(const double* in, float* out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}
__global__ void k_f2d(const float* in, double* out, size_t n, double beta) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = (beta == 0.0 ? 0.0 : beta * out[i]) + (double)in[i];
}

template <typename T>
void fill(Engine& E, T* p, T v, size_t n) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(256), 0, E.stream, p, v, n);
    ADC_HIP(hipGetLastError());
}
template <typename T>
void axpy(Engine& E, T a, const T* x, T* y, size_t n) {
    if (!n) return;
    hipLaunchKernelGGL(k_axpy<T>, dim3(grid_for(n)), dim3(256), 0, E.stream, a, x, y, n);
    ADC_HIP(hipGetLastError());
}
void convert_d2f(Engine& E, const double* in, float* out, size_t n) {
    if (!n) return;
    hipLaunchKernelGGL(k_d2f, dim3(grid_for(n)), dim3(256), 0, E.stream, in, out, n);
    ADC_HIP(hipGetLastError());
}
void convert_f2d(Engine& E, const float* in, double* out, size_t n, double beta) {
    if (!n) return;
    hipLaunchKernelGGL(k_f2d, dim3(grid_for(n)), dim3(256), 0, E.stream, in, out, n, beta);
    ADC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// contraction over sliced views, bounded temporaries
// ---------------------------------------------------------------------------
// out[sum_k idx_k ostr_k] = in[o] for the contiguous input (row-major over dim)
template <typename T>
__global__ void k_scatter(const T* __restrict__ in, T* __restrict__ out, PermArgs a,
                          long long total) {
    for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < total;
         o += (long long)gridDim.x * blockDim.x) {
        long long r = o, off = 0;
        for (int k = a.nd - 1; k >= 0; --k) {
            long long q = r / a.dim[k];
            off += (r - q * a.dim[k]) * a.istr[k];
            r = q;
        }
        out[off] = in[o];
    }
}

namespace {

// An operand as seen by a sliced contraction: its letters, the tensor's full
// row-major strides, the extent of each axis inside the slice, and the
// element offset of the slice's first element.
struct SView {
    std::string s;
    long long str[8], n[8];
    long long off = 0;
    long long size() const {
        long long z = 1;
        for (size_t k = 0; k < s.size(); ++k) z *= n[k];
        return z;
    }
    bool contiguous() const {
        long long st = 1;
        for (int k = (int)s.size() - 1; k >= 0; --k) {
            if (n[k] > 1 && str[k] != st) return false;
            st *= n[k];
        }
        return true;
    }
};

SView make_view(const Engine& E, const char* s, const std::vector<Slice>& sl) {
    SView v;
    v.s = s;
    const int nd = (int)v.s.size();
    ADC_REQUIRE(nd <= 8, "sliced contraction: rank > 8");
    long long st = 1;
    for (int k = nd - 1; k >= 0; --k) {
        v.str[k] = st;
        v.n[k] = E.ext.of(v.s[k]);
        st *= v.n[k];
    }
    for (const Slice& x : sl)
        for (int k = 0; k < nd; ++k)
            if (v.s[k] == x.c) {
                v.off += x.lo * v.str[k];
                v.n[k] = x.n;
            }
    return v;
}

PermArgs view_args(const SView& v) {
    PermArgs a;
    a.nd = (int)v.s.size();
    for (int k = 0; k < a.nd; ++k) {
        a.dim[k] = v.n[k];
        a.istr[k] = v.str[k];
    }
    return a;
}

}  // namespace

template <typename T>
static void ctr_leaf(Engine& E, T alpha, const SView& va, const T* A, const SView& vb, const T* B,
                     T beta, const SView& vc, T* C) {
    // letters whose slice is shorter than the tensor's extent get placeholder
    // names with the slice's extent (the same letter is sliced alike everywhere)
    std::map<char, char> ren;
    std::map<char, long long> saved;
    const char pool[] = "0123456789!#$%&*+-./:;<=>?";
    int next = 0;
    auto rename = [&](const SView& v) {
        std::string out = v.s;
        for (size_t k = 0; k < v.s.size(); ++k) {
            const char c = v.s[k];
            if (v.n[k] == E.ext.of(c) && !ren.count(c)) continue;
            if (!ren.count(c)) {
                ADC_REQUIRE(pool[next] != 0, "sliced contraction: too many sliced letters");
                ren[c] = pool[next++];
            }
            out[k] = ren[c];
        }
        return out;
    };
    // first pass: decide renamings from every view, then build the strings
    rename(va);
    rename(vb);
    rename(vc);
    const std::string sa = rename(va), sb = rename(vb), sc = rename(vc);
    for (auto& kv : ren) {
        long long n = -1;
        for (const SView* v : {&va, &vb, &vc})
            for (size_t k = 0; k < v->s.size(); ++k)
                if (v->s[k] == kv.first) n = v->n[k];
        auto it = E.ext.extra.find(kv.second);
        if (it != E.ext.extra.end()) saved[kv.second] = it->second;
        E.ext.extra[kv.second] = n;
    }
    struct Restore {
        Engine& e;
        std::map<char, char>& r;
        std::map<char, long long>& s;
        ~Restore() {
            for (auto& kv : r) e.ext.extra.erase(kv.second);
            for (auto& kv : s) e.ext.extra[kv.first] = kv.second;
        }
    } restore{E, ren, saved};
    auto gathered = [&](const SView& v, const T* p, int slot) -> const T* {
        if (v.contiguous()) return p + v.off;
        T* tmp = (T*)E.scratch.get(slot, sizeof(T) * v.size());
        const long long total = v.size();
        hipLaunchKernelGGL(k_permute<T>, dim3(grid_for(total)), dim3(256), 0, E.stream,
                           p + v.off, tmp, view_args(v), total, T(1), T(0));
        ADC_HIP(hipGetLastError());
        return tmp;
    };
    const T* Ap = gathered(va, A, 60);
    const T* Bp = gathered(vb, B, 61);
    if (vc.contiguous()) {
        ctr<T>(E, alpha, sa.c_str(), Ap, sb.c_str(), Bp, beta, sc.c_str(), C + vc.off);
        return;
    }
    T* Ct = beta == T(0) ? (T*)E.scratch.get(62, sizeof(T) * vc.size())
                         : const_cast<T*>(gathered(vc, C, 62));
    ctr<T>(E, alpha, sa.c_str(), Ap, sb.c_str(), Bp, beta, sc.c_str(), Ct);
    const long long total = vc.size();
    hipLaunchKernelGGL(k_scatter<T>, dim3(grid_for(total)), dim3(256), 0, E.stream, Ct,
                       C + vc.off, view_args(vc), total);
    ADC_HIP(hipGetLastError());
}

template <typename T>
void ctr_sliced(Engine& E, T alpha, const char* sa, const T* A, const char* sb, const T* B, T beta,
                const char* sc, T* C, const std::vector<Slice>& sl, long long budget) {
    if (budget <= 0) budget = E.slice_budget;
    const SView va = make_view(E, sa, sl), vb = make_view(E, sb, sl), vc = make_view(E, sc, sl);
    const SView* big = &va;
    for (const SView* v : {&vb, &vc})
        if (v->size() > big->size()) big = v;
    if (big->size() <= budget || va.size() == 0 || vb.size() == 0 || vc.size() == 0) {
        ctr_leaf<T>(E, alpha, va, A, vb, B, beta, vc, C);
        return;
    }
    // split the largest view along its longest axis: a free letter gives
    // disjoint output slices, a summed one partial sums added in block order
    int kbest = -1;
    for (size_t k = 0; k < big->s.size(); ++k)
        if (big->n[k] > 1 && (kbest < 0 || big->n[k] > big->n[kbest])) kbest = (int)k;
    ADC_REQUIRE(kbest >= 0, "sliced contraction: nothing to split");
    const char c = big->s[kbest];
    long long lo0 = 0;
    for (const Slice& x : sl)
        if (x.c == c) lo0 = x.lo;
    const long long n = big->n[kbest];
    const long long parts = std::min(n, (big->size() + budget - 1) / budget);
    const long long nb = (n + parts - 1) / parts;
    const bool summed = strchr(sc, c) == nullptr;
    for (long long b = 0; b < n; b += nb) {
        std::vector<Slice> s2;
        for (const Slice& x : sl)
            if (x.c != c) s2.push_back(x);
        s2.push_back({c, lo0 + b, std::min(nb, n - b)});
        ctr_sliced<T>(E, alpha, sa, A, sb, B, (summed && b > 0) ? T(1) : beta, sc, C, s2, budget);
    }
}

template void ctr_sliced<double>(Engine&, double, const char*, const double*, const char*,
                                 const double*, double, const char*, double*,
                                 const std::vector<Slice>&, long long);

template void ctr<double>(Engine&, double, const char*, const double*, const char*, const double*,
                          double, const char*, double*);
template void ctr<float>(Engine&, float, const char*, const float*, const char*, const float*,
                         float, const char*, float*);
template void permute<double>(Engine&, double, const char*, const double*, double, const char*,
                              double*);
template void permute<float>(Engine&, float, const char*, const float*, float, const char*, float*);
template void fill<double>(Engine&, double*, double, size_t);
template void fill<float>(Engine&, float*, float, size_t);
template void fill<int>(Engine&, int*, int, size_t);
template void axpy<double>(Engine&, double, const double*, double*, size_t);
template void axpy<float>(Engine&, float, const float*, float*, size_t);

}  // namespace adc
