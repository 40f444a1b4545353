// sigma = M_Z X (step 4 of Sec. III.A) for a block of vectors.
//
// The spin-adapted rows of Eqs. 36-37 act on Y = S^{-1/2} Z; the result is
// mapped back with S^{1/2} (both are 2x2 transforms on each (pq, qp) pair,
// applied by the LDS-tiled pair kernel).  Working layouts per vector z:
//   EA: Y1[z][a], Y2[z][i][a][b] = Y_abi   (a: attached alpha particle)
//   IP: Y1[z][i], Y2[z][a][i][j] = Y_ija   (i: removed alpha hole)
#include "context.hpp"

#include <algorithm>
#include <array>
#include <cmath>

namespace adc {

static const double SQ3 = 1.7320508075688772;
static const double AL = 0.5 * (1.0 + SQ3), BE = 0.5 * (1.0 - SQ3);                  // S^{+1/2}
static const double ALI = 0.5 * (1.0 + 1.0 / SQ3), BEI = 0.5 * (1.0 - 1.0 / SQ3);    // S^{-1/2}

enum Slot { S_Y1 = 10, S_Y2, S_S1, S_S2, S_W, S_U, S_T1, S_T2, S_T3, S_T4 };

template <typename T>
struct Views {
    const T *Boo, *Bov, *Bvo, *Bvv, *M11, *ovov, *oovv, *ooov, *oooo, *t, *tt, *gam, *Om, *Pi;
};

// HIP events around the particle-particle (hole-hole) kernels when timing is on
struct PPTimer {
    Engine& E;
    hipEvent_t a = nullptr, b = nullptr;
    explicit PPTimer(Engine& e) : E(e) {
        if (!E.timing) return;
        ADC_HIP(hipEventCreate(&a));
        ADC_HIP(hipEventCreate(&b));
        ADC_HIP(hipEventRecord(a, E.stream));
    }
    void stop() {
        if (!a) return;
        ADC_HIP(hipEventRecord(b, E.stream));
        ADC_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        ADC_HIP(hipEventElapsedTime(&ms, a, b));
        E.pp_ms += ms;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        a = b = nullptr;
    }
    ~PPTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

template <typename T>
static T* slot(Engine& E, int s, size_t n) {
    return (T*)E.scratch.get(s, n * sizeof(T));
}

// S1 = M11 Y1: the precomputed block, or applied on the fly (FP64)
template <typename T>
static void apply_11(adc_ctx* c, const T* M11, const T* Y1, T* S1, int nvec) {
    Engine& E = c->E;
    const bool ea = c->kind == ADC_EA;
    if (!c->m11_fly) {
        if (ea)
            ctr<T>(E, T(1), "ab", M11, "zb", Y1, T(0), "za", S1);
        else
            ctr<T>(E, T(1), "ij", M11, "zj", Y1, T(0), "zi", S1);
        return;
    }
    if constexpr (sizeof(T) == 8) {
        m11_fly(c, Y1, S1, nvec);
    } else {
        const size_t n = (size_t)nvec * c->n1;
        double* y = (double*)E.scratch.get(96, n * sizeof(double));
        double* s = (double*)E.scratch.get(97, n * sizeof(double));
        convert_f2d(E, Y1, y, n, 0.0);
        m11_fly(c, y, s, nvec);
        convert_d2f(E, s, S1, n);
    }
}

// first-order coupling, zeroth-order diagonal and the 11 block (ADC(2) and up)
template <typename T>
static void sigma_adc2_terms(adc_ctx* c, const Views<T>& v, const T* Y1, const T* Y2, T* S1, T* S2,
                             int nvec) {
    Engine& E = c->E;
    const long long Q = c->Q;
    if (c->kind == ADC_EA) {
        const int V = c->V;
        apply_11<T>(c, v.M11, Y1, S1, nvec);   // 11 block
        // 12: sigma_a += sum_bcj Y_bcj [(jb|ac) - 2 (jc|ab)]
        T* W = slot<T>(E, S_W, (size_t)nvec * V * Q);
        ctr<T>(E, T(1), "zjbc", Y2, "jbQ", v.Bov, T(0), "zcQ", W);
        ctr<T>(E, T(-2), "zjcb", Y2, "jbQ", v.Bov, T(1), "zcQ", W);
        ctr<T>(E, T(1), "acQ", v.Bvv, "zcQ", W, T(1), "za", S1);
        // 21: sigma_abi -= sum_c Y_c (ac|bi)
        T* U = slot<T>(E, S_U, (size_t)nvec * V * Q);
        ctr<T>(E, T(1), "zc", Y1, "acQ", v.Bvv, T(0), "azQ", U);
        ctr<T>(E, T(-1), "azQ", U, "ibQ", v.Bov, T(0), "ziab", S2);
        // 22, zeroth order: (e_a + e_b - e_i) Y_abi
        zeroth_order<T>(E, Y2, S2, nvec, c->O, V, c->eo.p, c->ev.p, -1.0, 1.0);
    } else {
        const int O = c->O;
        apply_11<T>(c, v.M11, Y1, S1, nvec);   // 11 block
        // 12: sigma_i += sum_jkb Y_jkb [(ki|jb) - 2 (kb|ji)]
        T* W = slot<T>(E, S_W, (size_t)nvec * O * Q);
        ctr<T>(E, T(1), "zbjk", Y2, "bjQ", v.Bvo, T(0), "zkQ", W);
        ctr<T>(E, T(-2), "zbkj", Y2, "bjQ", v.Bvo, T(1), "zkQ", W);
        ctr<T>(E, T(1), "kiQ", v.Boo, "zkQ", W, T(1), "zi", S1);
        // 21: sigma_ija -= sum_k Y_k (ki|aj)
        T* U = slot<T>(E, S_U, (size_t)nvec * O * Q);
        ctr<T>(E, T(1), "zk", Y1, "kiQ", v.Boo, T(0), "ziQ", U);
        ctr<T>(E, T(-1), "ziQ", U, "jaQ", v.Bov, T(0), "zaij", S2);
        // 22, zeroth order: (e_a - e_i - e_j) Y_ija
        zeroth_order<T>(E, Y2, S2, nvec, c->V, O, c->ev.p, c->eo.p, 1.0, -1.0);
    }
}

// second-order coupling and first-order 2p1h-2p1h terms of EA-ADC(3)
// (the particle-particle term is applied separately, in the Z basis)
template <typename T>
static void sigma_adc3_ea_terms(adc_ctx* c, const Views<T>& v, const T* Y1, const T* Y2, T* S1,
                                T* S2, int nvec) {
    Engine& E = c->E;
    const long long O = c->O, V = c->V, Q = c->Q;
    const size_t n4 = (size_t)nvec * O * V * V;
    const T* U = (const T*)E.scratch.get(S_U, 0);   // U[a][z][Q] = sum_c Bvv[a][c][Q] Y_c
    T* X1 = slot<T>(E, S_T1, std::max(n4, (size_t)(nvec * O * O * O)));
    T* X2 = slot<T>(E, S_T2, n4);
    T* X3 = slot<T>(E, S_T3, n4);
    T* W = slot<T>(E, S_W, (size_t)(nvec * std::max(O, V) * Q));
    // sigma_a: -Y_bcj t_kl^bc [2 (jl|ak) - (jk|al)]
    ctr<T>(E, T(1), "zjbc", Y2, "klbc", v.t, T(0), "zjkl", X1);
    ctr<T>(E, T(-2), "zjkl", X1, "jlka", v.ooov, T(1), "za", S1);
    ctr<T>(E, T(1), "zjkl", X1, "jkla", v.ooov, T(1), "za", S1);
    // sigma_a: (Y_baj - 2 Y_abj) Gamma_jb
    ctr<T>(E, T(1), "zjba", Y2, "jb", v.gam, T(1), "za", S1);
    ctr<T>(E, T(-2), "zjab", Y2, "jb", v.gam, T(1), "za", S1);
    // A~ = t~_jk^cd Y_bcj, B~ = t~_jk^cd Y_cbj, C~ = t~_jk^dc Y_cbj   ([z][b][k][d])
    //   F1 = -2 A~ + B~ -> (dk|ab),  F2 = A~ + C~ -> (db|ak)
    ctr<T>(E, T(1), "zjbc", Y2, "jkcd", v.tt, T(0), "zbkd", X1);        // A~
    ctr<T>(E, T(1), "zjcb", Y2, "jkcd", v.tt, T(0), "zbkd", X2);        // B~
    ctr<T>(E, T(1), "zjcb", Y2, "jkdc", v.tt, T(0), "zbkd", X3);        // C~
    axpy<T>(E, T(-2), X1, X2, n4);                                      // X2 = F1
    axpy<T>(E, T(1), X1, X3, n4);                                       // X3 = F2
    ctr<T>(E, T(1), "zbkd", X2, "kdQ", v.Bov, T(0), "zbQ", W);
    ctr<T>(E, T(1), "abQ", v.Bvv, "zbQ", W, T(1), "za", S1);
    ctr<T>(E, T(1), "zbkd", X3, "bdQ", v.Bvv, T(0), "zkQ", W);
    ctr<T>(E, T(1), "zkQ", W, "kaQ", v.Bov, T(1), "za", S1);
    // sigma_abi from Y1 (second order)
    ctr<T>(E, T(-1), "za", Y1, "ib", v.gam, T(1), "ziab", S2);
    ctr<T>(E, T(1), "zc", Y1, "likc", v.ooov, T(0), "zkli", X1);
    ctr<T>(E, T(-1), "zkli", X1, "klab", v.t, T(1), "ziab", S2);
    ctr<T>(E, T(1), "azQ", U, "kdQ", v.Bov, T(0), "zakd", X1);          // R = (ac|kd) Y_c
    ctr<T>(E, T(-1), "zakd", X1, "ikbd", v.tt, T(1), "ziab", S2);
    ctr<T>(E, T(1), "zc", Y1, "kcQ", v.Bov, T(0), "zkQ", W);
    ctr<T>(E, T(1), "zkQ", W, "adQ", v.Bvv, T(0), "zakd", X1);          // R' = (kc|ad) Y_c
    ctr<T>(E, T(1), "zakd", X1, "ikbd", v.t, T(1), "ziab", S2);
    ctr<T>(E, T(1), "zbkd", X1, "ikda", v.t, T(1), "ziab", S2);
    // first-order 2p1h-2p1h: (2 Y_acj - Y_caj)(jc|ib) - Y_acj (ji|bc) - Y_cbj (ji|ac)
    pair_transform<T, T>(E, Y2, (long long)(O * V * V), 0, X1, (long long)(O * V * V), 0, nvec, O,
                      (int)V, 2.0, -1.0, 0.0);
    ctr<T>(E, T(1), "zjac", X1, "jcib", v.ovov, T(1), "ziab", S2);
    ctr<T>(E, T(-1), "zjac", Y2, "jibc", v.oovv, T(1), "ziab", S2);
    ctr<T>(E, T(-1), "zjcb", Y2, "jiac", v.oovv, T(1), "ziab", S2);
}

// second-order coupling and first-order 2h1p-2h1p terms of IP-ADC(3)
// (the hole-hole term is applied separately, in the Z basis)
template <typename T>
static void sigma_adc3_ip_terms(adc_ctx* c, const Views<T>& v, const T* Y1, const T* Y2, T* S1,
                                T* S2, int nvec) {
    Engine& E = c->E;
    const long long O = c->O, V = c->V;
    const size_t n3 = (size_t)(nvec * O * O * V);
    T* X1 = slot<T>(E, S_T1, n3);
    T* X2 = slot<T>(E, S_T2, n3);
    // sigma_i: A~[j][l][c] = Y_jkb t~_kl^bc -> (jl|ic) - 2 (ji|lc)
    ctr<T>(E, T(1), "zbjk", Y2, "klbc", v.tt, T(0), "zjlc", X1);
    ctr<T>(E, T(1), "zjlc", X1, "jlic", v.ooov, T(1), "zi", S1);
    ctr<T>(E, T(-2), "zjlc", X1, "jilc", v.ooov, T(1), "zi", S1);
    //   Y_jkb t~_jl^bc (ki|lc) + Y_jkb t~_jl^cb (kl|ic)
    ctr<T>(E, T(1), "zbjk", Y2, "jlbc", v.tt, T(0), "zklc", X1);
    ctr<T>(E, T(1), "zklc", X1, "kilc", v.ooov, T(1), "zi", S1);
    ctr<T>(E, T(1), "zbjk", Y2, "jlcb", v.tt, T(0), "zklc", X1);
    ctr<T>(E, T(1), "zklc", X1, "klic", v.ooov, T(1), "zi", S1);
    //   Y_jkb Omega[i][k][j][b] + (2 Y_ijb - Y_jib) Gamma_jb
    ctr<T>(E, T(1), "zbjk", Y2, "ikjb", v.Om, T(1), "zi", S1);
    ctr<T>(E, T(2), "zbij", Y2, "jb", v.gam, T(1), "zi", S1);
    ctr<T>(E, T(-1), "zbji", Y2, "jb", v.gam, T(1), "zi", S1);
    // sigma_ija from Y1 (second order)
    ctr<T>(E, T(1), "zi", Y1, "ja", v.gam, T(1), "zaij", S2);
    ctr<T>(E, T(1), "zk", Y1, "kilb", v.ooov, T(0), "zilb", X1);      // Z  = Y_k (ki|lb)
    ctr<T>(E, T(-1), "zilb", X1, "jlab", v.tt, T(1), "zaij", S2);
    ctr<T>(E, T(1), "zk", Y1, "likb", v.ooov, T(0), "zilb", X1);      // Z' = Y_k (li|kb)
    ctr<T>(E, T(1), "zilb", X1, "jlab", v.t, T(1), "zaij", S2);
    ctr<T>(E, T(1), "zjlb", X1, "ilba", v.t, T(1), "zaij", S2);
    ctr<T>(E, T(-1), "zk", Y1, "kjia", v.Pi, T(1), "zaij", S2);
    // first-order 2h1p-2h1p: (2 Y_ikb - Y_kib)(kb|ja) - Y_ikb (kj|ab) - Y_kjb (ki|ab)
    pair_transform<T, T>(E, Y2, (long long)(V * O * O), 0, X2, (long long)(V * O * O), 0, nvec, V,
                      (int)O, 2.0, -1.0, 0.0);
    ctr<T>(E, T(1), "zbik", X2, "kbja", v.ovov, T(1), "zaij", S2);
    ctr<T>(E, T(-1), "zbik", Y2, "kjab", v.oovv, T(1), "zaij", S2);
    ctr<T>(E, T(-1), "zbkj", Y2, "kiab", v.oovv, T(1), "zaij", S2);
}


template <typename T>
static Views<T> views(adc_ctx* c, bool big = true);

template <>
Views<double> views<double>(adc_ctx* c, bool big) {
    if (big) ensure_tt(c);
    return Views<double>{c->Boo.p,  c->Bov.p,  c->Bvo.p,  c->Bvv.p, c->M11.p,
                         c->ovov.p, c->oovv.p, c->ooov.p, c->oooo.p, c->t.p,
                         c->tt.p,   c->gam.p,  c->Om.p,   c->Pi.p};
}

template <>
Views<float> views<float>(adc_ctx* c, bool big) {
    build_mixed(c, big);
    return Views<float>{c->fBoo.p,  c->fBov.p,  c->fBvo.p,  c->fBvv.p, c->fM11.p,
                        c->fovov.p, c->foovv.p, c->fooov.p, c->foooo.p, c->ft.p,
                        c->ftt.p,   c->fgam.p,  c->fOm.p,   c->fPi.p};
}

// Precision levels of sigma: FP64; FP32 storage with BF16 products (the big
// operands of the arranged EA products and of the particle-particle term in
// BF16); FP32 storage with FP32 products.  T is the storage of the vectors
// and most operands, TB that of the large product operands.

// Operands of the arranged EA path (ea_layout.hip); H = t~ B_ov and BH = B_ov + H
// fold two of the t~ products into products over Naux
template <typename T, typename TB>
struct EaOps {
    const TB *ttT1, *ttT2, *tT1, *tD, *oovvT, *tT, *ovov;
    const T *G, *Bvo, *H, *BH;
};

static EaOps<double, double> ea_ops(adc_ctx* c, double*, double*) {
    auto& L = c->eal;
    return {L.ttT1.p, L.ttT2.p, L.tT1.p, L.tD.p, L.oovvT.p, L.tT.p, c->ovov.p,
            L.G.p,    c->Bvo.p, L.H.p,   L.BH.p};
}
static EaOps<float, bf16_t> ea_ops(adc_ctx* c, float*, bf16_t*) {
    auto& L = c->eal;
    return {L.httT1.p, L.httT2.p, L.htT1.p, L.htD.p, L.hoovvT.p, L.htT.p, L.hovov.p,
            L.fG.p,    c->fBvo.p, L.fH.p,   L.fBH.p};
}
static EaOps<float, float> ea_ops(adc_ctx* c, float*, float*) {
    auto& L = c->eal;
    return {L.fttT1.p, L.fttT2.p, L.ftT1.p, L.ftD.p, L.foovvT.p, L.ftT.p, c->fovov.p,
            L.fG.p,    c->fBvo.p, L.fH.p,   L.fBH.p};
}

// sigma precision level of a (T, TB) pair: 0 FP64, 1 BF16 products, 2 FP32 products
template <typename T, typename TB>
constexpr int level_of() {
    return sizeof(T) == 8 ? 0 : sizeof(TB) == 2 ? 1 : 2;
}

static GemmOut omap(long long rsplit, long long rs1, long long rs2, long long csplit, long long cs1,
                    long long cs2) {
    GemmOut o;
    o.rsplit = rsplit;
    o.rs1 = rs1;
    o.rs2 = rs2;
    o.csplit = csplit;
    o.cs1 = cs1;
    o.cs2 = cs2;
    return o;
}

enum ArrSlot { A_P1 = 40, A_P2, A_PM = 43, A_DW, A_W, A_X1, A_F2, A_W2, A_X, A_RP = 51, A_WK,
               A_SLICE = 70 };

// ---------------------------------------------------------------------------
// blocked products: arranged operands built per call, one block at a time
// ---------------------------------------------------------------------------
// out[x][y][z][w] (x < n) = al src[(x0+x) s0 + y s1 + z s2 + w s3]
//                         + be src[(x0+x) r0 + y r1 + z r2 + w r3]
// (the block of an operand rearranged from a resident FP64 tensor, rounded to
// the product's storage type: BF16 through FP32, as the resident copies are)
struct ArrSpec {
    const double* src;
    long long e1, e2, e3;
    long long s[4], r[4];
    double al, be;
};

template <typename TB>
__device__ __forceinline__ TB narrow_to(double v) {
    if constexpr (sizeof(TB) == 2)
        return (TB)(float)v;
    else
        return (TB)v;
}

template <typename TB>
__global__ void k_arrange(ArrSpec a, long long x0, long long total, TB* __restrict__ out) {
    for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < total;
         o += (long long)gridDim.x * blockDim.x) {
        long long q = o;
        const long long w = q % a.e3;
        q /= a.e3;
        const long long z = q % a.e2;
        q /= a.e2;
        const long long y = q % a.e1;
        const long long x = q / a.e1 + x0;
        double v = a.al * a.src[x * a.s[0] + y * a.s[1] + z * a.s[2] + w * a.s[3]];
        if (a.be != 0.0) v += a.be * a.src[x * a.r[0] + y * a.r[1] + z * a.r[2] + w * a.r[3]];
        out[o] = narrow_to<TB>(v);
    }
}

// The same arrangement when one term reads its second index (y) with unit
// stride and its last index (w) with a large one: a 32x32 (y, w) tile of that
// term is read along y (coalesced), transposed through LDS and written along
// w; the other term (if any) has unit stride in w and is read directly.
// Tiles: grid.x over (y, w) tiles, grid.y over z, grid.z over the block's
// leading indices.
struct ArrTerm {
    long long s[4];
    double al;
};
template <typename TB>
__global__ void k_arrange_tiled(const double* __restrict__ src, ArrTerm tr, ArrTerm dr,
                                bool direct, long long e1, long long e2, long long e3,
                                long long x0, int ntw, TB* __restrict__ out) {
    __shared__ double tile[32][33];
    const int ty = threadIdx.y, tx = threadIdx.x;   // 8 x 32
    const long long y0 = (long long)(blockIdx.x / ntw) * 32, w0 = (long long)(blockIdx.x % ntw) * 32;
    const long long z = blockIdx.y, xl = blockIdx.z, x = x0 + xl;
    const double* base = src + x * tr.s[0] + z * tr.s[2];
    for (int r = ty; r < 32; r += 8) {
        const long long w = w0 + r, y = y0 + tx;
        tile[r][tx] = (w < e3 && y < e1) ? base[y * tr.s[1] + w * tr.s[3]] : 0.0;
    }
    __syncthreads();
    const double* dbase = src + x * dr.s[0] + z * dr.s[2];
    for (int r = ty; r < 32; r += 8) {
        const long long y = y0 + r, w = w0 + tx;
        if (y >= e1 || w >= e3) continue;
        double v = tr.al * tile[tx][r];
        if (direct) v += dr.al * dbase[y * dr.s[1] + w * dr.s[3]];
        out[((xl * e1 + y) * e2 + z) * e3 + w] = narrow_to<TB>(v);
    }
}

static ArrSpec arr(const double* src, long long e1, long long e2, long long e3,
                   std::array<long long, 4> s, double al = 1.0,
                   std::array<long long, 4> r = {0, 0, 0, 0}, double be = 0.0) {
    ArrSpec a;
    a.src = src;
    a.e1 = e1;
    a.e2 = e2;
    a.e3 = e3;
    for (int k = 0; k < 4; ++k) {
        a.s[k] = s[k];
        a.r[k] = r[k];
    }
    a.al = al;
    a.be = be;
    return a;
}

// One NT product whose operand A (arranged_a) or B is the arranged tensor of
// `nlead` leading indices, each of e1 rows of K = e2 e3 elements; run in
// blocks of leading indices, each block of the result stored at C + x0 c_off
// through the same output map.
template <typename TB, typename TO>
static void blocked_nt(adc_ctx* c, bool arranged_a, long long M_or_N, const ArrSpec& a,
                       long long nlead, double alpha, const TB* other, long long ld_other,
                       double beta, TO* C, GemmOut map, long long c_off) {
    Engine& E = c->E;
    const long long rows = a.e1, K = a.e2 * a.e3;
    const long long per = rows * K * (long long)sizeof(TB);
    const long long nb =
        std::max<long long>(1, std::min<long long>(nlead, E.slice_budget * 8 / per));
    TB* sl = (TB*)E.scratch.get(A_SLICE, (size_t)(nb * rows * K) * sizeof(TB));
    for (long long x0 = 0; x0 < nlead; x0 += nb) {
        const long long n = std::min(nb, nlead - x0);
        const long long total = n * rows * K;
        long long g = (total + 255) / 256;
        g = std::max<long long>(1, std::min<long long>(g, 1LL << 20));
        // a term with unit stride in y and not in w goes through the LDS
        // transpose (the other term, if any, must have unit stride in w)
        const bool t_s = a.s[1] == 1 && a.s[3] != 1 && (a.be == 0.0 || a.r[3] == 1);
        const bool t_r = !t_s && a.be != 0.0 && a.r[1] == 1 && a.r[3] != 1 && a.s[3] == 1;
        if ((t_s || t_r) && a.e2 <= 65535 && n <= 65535) {
            ArrTerm tr, dr;
            for (int k = 0; k < 4; ++k) {
                tr.s[k] = t_s ? a.s[k] : a.r[k];
                dr.s[k] = t_s ? a.r[k] : a.s[k];
            }
            tr.al = t_s ? a.al : a.be;
            dr.al = t_s ? a.be : a.al;
            const long long nty = (rows + 31) / 32, ntw = (a.e3 + 31) / 32;
            ADC_REQUIRE(nty * ntw < (1LL << 31), "arrange: too many tiles");
            hipLaunchKernelGGL(k_arrange_tiled<TB>, dim3((unsigned)(nty * ntw), (unsigned)a.e2,
                                                         (unsigned)n),
                               dim3(32, 8), 0, E.stream, a.src, tr, dr, a.be != 0.0, rows, a.e2,
                               a.e3, x0, (int)ntw, sl);
        } else {
            hipLaunchKernelGGL(k_arrange<TB>, dim3((unsigned)g), dim3(256), 0, E.stream, a, x0,
                               total, sl);
        }
        ADC_HIP(hipGetLastError());
        if (arranged_a)
            gemm_map<TB, TO>(E, false, true, n * rows, M_or_N, K, alpha, sl, K, other, ld_other,
                             beta, C + x0 * c_off, map);
        else
            gemm_map<TB, TO>(E, false, true, M_or_N, n * rows, K, alpha, other, ld_other, sl, K,
                             beta, C + x0 * c_off, map);
    }
}

// EA sigma (ADC(2) terms and, for ADC(3), the second-order coupling and the
// first-order 2p1h-2p1h terms; the particle-particle term is applied
// separately) with every large contraction one NT product of arranged
// operands.  The contractions are those of the generic path term by term,
// except two t~ products regrouped through the resident
// H[i][b][Q] = sum_kd t~_ik^bd (kd|Q) (t~ is symmetric under the exchange of
// its (occupied, virtual) pairs):
//   D[z][x][j][y] = Y_yxj - 2 Y_xyj   carries (Y_bcj - 2 Y_cbj) of the
//                   first-order coupling and (Y_baj - 2 Y_abj) Gamma_jb,
//   F1 = D t~  only feeds the (jb|Q) product: (D + F1) B_ov = D (B_ov + H),
//   R t~ with R = (ac|kd) Y_c is U H^T, U = sum_c Y_c (ac|Q),
//   F2 = A~ + C~  is written as [z][k][b][d] for its (bd|Q) product,
//   S2 gets every (z,a)x(i,b) and (i,a)x(z,b) product through an output map.
template <typename T, typename TB>
static void sigma_ea_arranged(adc_ctx* c, const T* Y1, const T* Y2, T* S1, T* S2, int nvec) {
    Engine& E = c->E;
    ea_layout_build(c, level_of<T, TB>());
    const bool blocked = c->eal.mode == 2;
    const Views<T> v = views<T>(c, !blocked);
    const long long Z = nvec, O = c->O, V = c->V, Q = c->Q;
    const long long OV = O * V, VV = V * V, OVV = O * VV;
    const size_t n4 = (size_t)(Z * OVV);
    const bool o3 = c->order == 3;

    apply_11<T>(c, v.M11, Y1, S1, nvec);   // 11 block
    // pair tensors of the trial vectors
    T* Dw = slot<T>(E, A_DW, n4);
    TB *P1 = nullptr, *P2 = nullptr, *Pm = nullptr;
    if (o3) {
        P1 = slot<TB>(E, A_P1, n4);
        P2 = slot<TB>(E, A_P2, n4);
        Pm = slot<TB>(E, A_PM, n4);
    }
    ea_pairs<T, TB>(E, Y2, nvec, (int)O, (int)V, P1, P2, (TB*)nullptr, Pm, Dw);
    // 21: sigma_abi = -sum_Q U[a][z][Q] (ib|Q),  U = sum_c Y_c (ac|Q)
    T* U = slot<T>(E, S_U, (size_t)(V * Z * Q));
    const bool host = c->bvv_host;   // B_vv rows staged from host memory per product
    const long long bvr = host ? std::max<long long>(1, bvv_chunk_rows(c, sizeof(T)) / V) : V;
    if (!host) {
        ctr<T>(E, T(1), "zc", Y1, "acQ", v.Bvv, T(0), "azQ", U);
    } else {
        for (long long a0 = 0; a0 < V; a0 += bvr) {
            const long long n = std::min(bvr, V - a0);
            E.ext.extra['A'] = n;
            ctr<T>(E, T(1), "zc", Y1, "AcQ", bvv_rows<T>(c, a0 * V, n * V, 72), T(0), "AzQ",
                   U + a0 * Z * Q);
        }
        E.ext.extra.erase('A');
    }
    const GemmOut S2_zaib = omap(V, OVV, V, V, VV, 1);    // rows (z,a), columns (i,b)
    const GemmOut S2_iazb = omap(V, VV, V, V, OVV, 1);    // rows (i,a), columns (z,b)
    gemm_map<T, T>(E, false, true, V * Z, OV, Q, -1.0, U, Q, v.Bov, Q, 0.0, S2,
                   omap(Z, V, OVV, V, VV, 1));
    // 22, zeroth order
    zeroth_order<T>(E, Y2, S2, nvec, O, (int)V, c->eo.p, c->ev.p, -1.0, 1.0);

    T* W = slot<T>(E, A_W, (size_t)(Z * V * Q));
    const T* BW = v.Bov;    // right operand of the (jb|Q) product
    if (o3) {
        const EaOps<T, TB> a = ea_ops(c, (T*)nullptr, (TB*)nullptr);
        BW = a.BH;
        // the arranged operands of the blocked path, from the resident FP64 t,
        // (ov|ov) and (oo|vv) (strides of t[j][k][c][d] = t_jk^cd: O V^2, V^2, V, 1)
        const double *t = c->t.p, *ovv = c->ovov.p, *oov = c->oovv.p;
        const long long s0 = OVV, s1 = VV;
        // t~_jk^cd as [k][d][j][c] and t~_jk^dc as [k][d][j][c]
        const ArrSpec tt1 = arr(t, V, O, V, {s1, 1, s0, V}, 2.0, {s1, V, s0, 1}, -1.0);
        const ArrSpec tt2 = arr(t, V, O, V, {s1, V, s0, 1}, 2.0, {s1, 1, s0, V}, -1.0);
        const ArrSpec t1 = arr(t, V, O, V, {s1, 1, s0, V});          // t_jk^cd [k][d][j][c]
        const ArrSpec tD = arr(t, V, O, V, {s0, 1, s1, V});          // t_ik^da [i][a][k][d]
        const ArrSpec oT = arr(oov, V, O, V, {s1, V, s0, 1});        // (ji|bc) [i][b][j][c]
        const ArrSpec tTa = arr(t, V, O, O, {V, 1, s0, s1});         // t_kl^ab [a][b][k][l]
        const ArrSpec ovI = arr(ovv, V, O, V, {s0, O * V, V, 1});    // (ov|ov) as it is
        const ArrSpec tI = arr(t, O, V, V, {s0, s1, V, 1});          // t as it is
        // sigma_a += sum_jb (Y_baj - 2 Y_abj) Gamma_jb
        gemm_map<T, T>(E, false, true, Z * V, 1, OV, 1.0, Dw, OV, v.gam, OV, 1.0, S1,
                       GemmOut::rowmajor(1));
        // sigma_a -= sum_jkl Y_bcj t_kl^bc [2 (jl|ka) - (jk|la)]
        T* X1 = slot<T>(E, A_X1, (size_t)(Z * O * O * O));
        if (!blocked || sizeof(T) == 8)
            gemm_map<T, T>(E, false, true, Z * O, O * O, VV, 1.0, Y2, VV,
                           blocked ? (const T*)c->t.p : v.t, VV, 0.0, X1, GemmOut::rowmajor(O * O));
        else
            blocked_nt<T, T>(c, false, Z * O, tI, O, 1.0, Y2, VV, 0.0, X1,
                             GemmOut::rowmajor(O * O), O);
        gemm_map<T, T>(E, false, true, Z, V, O * O * O, 1.0, X1, O * O * O, a.G, O * O * O, 1.0,
                       S1, GemmOut::rowmajor(V));
        // F2 = A~ + C~ as F2[z][k][b][d], then sigma_a += sum_kQ (sum_bd F2 (bd|Q)) (ka|Q)
        T* F2 = slot<T>(E, A_F2, n4);
        const GemmOut f2map = omap(V, OVV, V, V, VV, 1);
        if (blocked) {
            blocked_nt<TB, T>(c, false, Z * V, tt1, O, 1.0, P1, OV, 0.0, F2, f2map, VV);
            blocked_nt<TB, T>(c, false, Z * V, tt2, O, 1.0, P2, OV, 1.0, F2, f2map, VV);
        } else {
            gemm_map<TB, T>(E, false, true, Z * V, OV, OV, 1.0, P1, OV, a.ttT1, OV, 0.0, F2, f2map);
            gemm_map<TB, T>(E, false, true, Z * V, OV, OV, 1.0, P2, OV, a.ttT2, OV, 1.0, F2, f2map);
        }
        T* W2 = slot<T>(E, A_W2, (size_t)(Z * O * Q));
        if (!host)
            gemm_map<T, T>(E, false, false, Z * O, Q, VV, 1.0, F2, VV, v.Bvv, Q, 0.0, W2,
                           GemmOut::rowmajor(Q));
        else
            for (long long b0 = 0; b0 < V; b0 += bvr) {
                const long long n = std::min(bvr, V - b0);
                gemm_map<T, T>(E, false, false, Z * O, Q, n * V, 1.0, F2 + b0 * V, VV,
                               bvv_rows<T>(c, b0 * V, n * V, 72), Q, b0 == 0 ? 0.0 : 1.0, W2,
                               GemmOut::rowmajor(Q));
            }
        gemm_map<T, T>(E, false, true, Z, V, O * Q, 1.0, W2, O * Q, a.Bvo, O * Q, 1.0, S1,
                       GemmOut::rowmajor(V));
        // sigma_abi -= Y_a Gamma_ib
        gemm_map<T, T>(E, false, true, Z * V, OV, 1, -1.0, Y1, 1, v.gam, 1, 1.0, S2, S2_zaib);
        // sigma_abi -= sum_kl (sum_c Y_c (li|kc)) t_kl^ab, the inner sum stored [z][i][k][l]
        TB* X = slot<TB>(E, A_X, (size_t)(Z * O * O * O));
        gemm_map<T, TB>(E, false, true, Z, O * O * O, V, 1.0, Y1, V, v.ooov, V, 0.0, X,
                        omap(0, 0, O * O * O, O * O, 1, O));
        if (blocked)
            blocked_nt<TB, T>(c, false, Z * O, tTa, V, -1.0, X, O * O, 1.0, S2,
                              GemmOut::rowmajor(VV), V);
        else
            gemm_map<TB, T>(E, false, true, Z * O, VV, O * O, -1.0, X, O * O, a.tT, O * O, 1.0, S2,
                            GemmOut::rowmajor(VV));
        // sigma_abi -= sum_kd [(ac|kd) Y_c] t~_ik^bd = sum_Q U[a][z][Q] H[i][b][Q]
        gemm_map<T, T>(E, false, true, V * Z, OV, Q, -1.0, U, Q, a.H, Q, 1.0, S2,
                       omap(Z, V, OVV, V, VV, 1));
        // R'[z][a][k][d] = (kc|ad) Y_c:  sigma_abi += R' t_ik^bd + R'[z][b] t_ik^da
        T* Wk = slot<T>(E, A_WK, (size_t)(Z * O * Q));
        ctr<T>(E, T(1), "zc", Y1, "kcQ", v.Bov, T(0), "zkQ", Wk);
        TB* Rp = slot<TB>(E, A_RP, n4);
        if (!host)
            gemm_map<T, TB>(E, false, true, Z * O, VV, Q, 1.0, Wk, Q, v.Bvv, Q, 0.0, Rp,
                            omap(O, OVV, V, V, OV, 1));
        else
            for (long long a0 = 0; a0 < V; a0 += bvr) {
                const long long n = std::min(bvr, V - a0);
                gemm_map<T, TB>(E, false, true, Z * O, n * V, Q, 1.0, Wk, Q,
                                bvv_rows<T>(c, a0 * V, n * V, 72), Q, 0.0, Rp + a0 * OV,
                                omap(O, OVV, V, V, OV, 1));
            }
        if (blocked) {
            blocked_nt<TB, T>(c, false, Z * V, t1, O, 1.0, Rp, OV, 1.0, S2, S2_zaib, VV);
            blocked_nt<TB, T>(c, true, Z * V, tD, O, 1.0, Rp, OV, 1.0, S2, S2_iazb, VV);
            // first-order 2p1h-2p1h: (2 Y_acj - Y_caj)(jc|ib) - Y_acj (ji|bc) - Y_cbj (ji|ac)
            if (sizeof(TB) == 8)
                gemm_map<TB, T>(E, false, true, Z * V, OV, OV, 1.0, Pm, OV, (const TB*)ovv, OV,
                                1.0, S2, S2_zaib);
            else
                blocked_nt<TB, T>(c, false, Z * V, ovI, O, 1.0, Pm, OV, 1.0, S2, S2_zaib, VV);
            blocked_nt<TB, T>(c, false, Z * V, oT, O, -1.0, P1, OV, 1.0, S2, S2_zaib, VV);
            blocked_nt<TB, T>(c, true, Z * V, oT, O, -1.0, P2, OV, 1.0, S2, S2_iazb, VV);
        } else {
            gemm_map<TB, T>(E, false, true, Z * V, OV, OV, 1.0, Rp, OV, a.tT1, OV, 1.0, S2, S2_zaib);
            gemm_map<TB, T>(E, false, true, OV, Z * V, OV, 1.0, a.tD, OV, Rp, OV, 1.0, S2, S2_iazb);
            // first-order 2p1h-2p1h: (2 Y_acj - Y_caj)(jc|ib) - Y_acj (ji|bc) - Y_cbj (ji|ac)
            gemm_map<TB, T>(E, false, true, Z * V, OV, OV, 1.0, Pm, OV, a.ovov, OV, 1.0, S2, S2_zaib);
            gemm_map<TB, T>(E, false, true, Z * V, OV, OV, -1.0, P1, OV, a.oovvT, OV, 1.0, S2, S2_zaib);
            gemm_map<TB, T>(E, false, true, OV, Z * V, OV, -1.0, a.oovvT, OV, P2, OV, 1.0, S2, S2_iazb);
        }
    }
    // sigma_a += sum_cQ (ac|Q) W[z][c][Q],  W = sum_jb D[z][c][j][b] [(jb|Q) + H_jb^Q]
    // (ADC(2): no H)
    gemm_map<T, T>(E, false, false, Z * V, Q, OV, 1.0, Dw, OV, BW, Q, 0.0, W,
                   GemmOut::rowmajor(Q));
    if (!host)
        gemm_map<T, T>(E, false, true, Z, V, V * Q, 1.0, W, V * Q, v.Bvv, V * Q, 1.0, S1,
                       GemmOut::rowmajor(V));
    else
        for (long long a0 = 0; a0 < V; a0 += bvr) {
            const long long n = std::min(bvr, V - a0);
            gemm_map<T, T>(E, false, true, Z, n, V * Q, 1.0, W, V * Q,
                           bvv_rows<T>(c, a0 * V, n * V, 72), V * Q, 1.0, S1 + a0,
                           GemmOut::rowmajor(V));
        }
}

template <typename T, typename TB>
void sigma_block(adc_ctx* c, const double* X, double* Yout, int nvec) {
    Engine& E = c->E;
    E.ext.Z = nvec;
    const int n1 = c->n1;
    const long long nx = c->n2x;
    const int np = (int)c->n2p;
    const long long len2 = nx * np * np;
    const long long dim = c->dim;
    const bool arranged = ea_layout_use(c, level_of<T, TB>());
    Views<T> v = views<T>(c, !(arranged && c->eal.mode == 2));
    // FP32 contractions multiply in BF16 on the matrix cores in the mixed mode
    struct Bf16Scope {
        Engine& e;
        bool old;
        Bf16Scope(Engine& en, bool on) : e(en), old(en.bf16) { e.bf16 = on; }
        ~Bf16Scope() { e.bf16 = old; }
    } scope(E, level_of<T, TB>() == 1);

    T* Y1 = slot<T>(E, S_Y1, (size_t)nvec * n1);
    T* Y2 = slot<T>(E, S_Y2, (size_t)nvec * len2);
    T* S1 = slot<T>(E, S_S1, (size_t)nvec * n1);
    T* S2 = slot<T>(E, S_S2, (size_t)nvec * len2);

    // Y = S^{-1/2} Z
    copy_rows<double, T>(E, X, dim, 0, Y1, n1, 0, nvec, n1, 0.0);
    pair_transform<double, T>(E, X, dim, n1, Y2, len2, 0, nvec, nx, np, ALI, BEI, 0.0);

    const bool ea3 = c->order == 3 && c->kind == ADC_EA;
    const bool ip3 = c->order == 3 && c->kind == ADC_IP;
    if (arranged) {
        sigma_ea_arranged<T, TB>(c, Y1, Y2, S1, S2, nvec);
    } else {
        sigma_adc2_terms<T>(c, v, Y1, Y2, S1, S2, nvec);
        if (ea3) sigma_adc3_ea_terms<T>(c, v, Y1, Y2, S1, S2, nvec);
        if (ip3) sigma_adc3_ip_terms<T>(c, v, Y1, Y2, S1, S2, nvec);
    }

    // Z-basis result: S^{1/2} sigma_Y (+ the particle-particle term, which commutes
    // with the pair metric and acts on Z directly)
    copy_rows<T, double>(E, S1, n1, 0, Yout, dim, 0, nvec, n1, 0.0);
    double beta2 = 0.0;
    if (ea3) {
        using P = TB;
        const P* Bvv = c->bvv_host                ? nullptr   // staged from host memory
                       : level_of<T, TB>() == 0   ? (const P*)c->Bvv.p
                       : level_of<T, TB>() == 1 ? (const P*)c->hBvv.p
                                                : (const P*)c->fBvv.p;
        P* Zp = slot<P>(E, S_T4, (size_t)nvec * len2);
        T* Zv = slot<T>(E, S_T1, (size_t)nvec * len2);
        copy_rows<double, P>(E, X, dim, n1, Zp, len2, 0, nvec, len2, 0.0);
        PPTimer tm(E);
        vvvv_apply<P, T>(c, Bvv, Zp, Zv, (long long)nvec * c->O);
        tm.stop();
        copy_rows<T, double>(E, Zv, len2, 0, Yout, dim, n1, nvec, len2, 0.0);
        beta2 = 1.0;
    }
    if (ip3) {
        // hole-hole term sum_kl (ki|lj) Z_kla, commutes with the pair metric
        T* Zp = slot<T>(E, S_T4, (size_t)nvec * len2);
        T* Zv = slot<T>(E, S_T1, (size_t)nvec * len2);
        copy_rows<double, T>(E, X, dim, n1, Zp, len2, 0, nvec, len2, 0.0);
        PPTimer tm(E);
        ctr<T>(E, T(1), "kilj", v.oooo, "zakl", Zp, T(0), "zaij", Zv);
        tm.stop();
        copy_rows<T, double>(E, Zv, len2, 0, Yout, dim, n1, nvec, len2, 0.0);
        beta2 = 1.0;
    }
    pair_transform<T, double>(E, S2, len2, 0, Yout, dim, n1, nvec, nx, np, AL, BE, beta2);
}

void sigma_eager(adc_ctx* c, const double* X, double* Y, int nvec, int precision) {
    if (c->uhf)
        sigma_uhf(c, X, Y, nvec);
    else if (precision == 1)
        sigma_block<float, bf16_t>(c, X, Y, nvec);
    else if (precision == 2)
        sigma_block<float, float>(c, X, Y, nvec);
    else
        sigma_block<double, double>(c, X, Y, nvec);
}

void drop_graphs(adc_ctx* c) {
    for (auto& g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

// sigma replayed from a HIP graph.  The graph is captured over the internal
// buffers Xg -> Yg after an eager warm-up call with the same sizes (which
// allocates every scratch buffer and settles the GEMM autotuner, so the
// captured region holds kernel launches only); it is re-captured when one of
// the scratch buffers it uses has been reallocated or freed since.
static void sigma_graph(adc_ctx* c, const double* X, double* Y, int nvec, int precision) {
    Engine& E = c->E;
    // the null stream cannot be captured: use a blocking stream of the
    // context's own (default priority), ordered with null-stream work
    struct StreamScope {
        Engine& e;
        hipStream_t old;
        ~StreamScope() { e.stream = old; }
    } scope{E, E.stream};
    const bool own = !E.stream;
    if (own) {
        if (!c->gstream) ADC_HIP(hipStreamCreate(&c->gstream));
        if (!c->gdone) ADC_HIP(hipEventCreateWithFlags(&c->gdone, hipEventDisableTiming));
        E.stream = c->gstream;
    }
    const size_t bytes = (size_t)nvec * c->dim * sizeof(double);
    if (c->Xg.n < (size_t)nvec * c->dim) {
        drop_graphs(c);
        c->Xg.alloc((size_t)nvec * c->dim, &c->arena);
        c->Yg.alloc((size_t)nvec * c->dim, &c->arena);
    }
    ADC_HIP(hipMemcpyAsync(c->Xg.p, X, bytes, hipMemcpyDeviceToDevice, E.stream));
    adc_ctx::SigmaGraph* g = nullptr;
    for (auto& e : c->graphs)
        if (e.nvec == nvec && e.precision == precision) g = &e;
    if (g && g->exec && !E.scratch.still_valid(g->slots)) {
        (void)hipGraphExecDestroy(g->exec);
        (void)hipGraphDestroy(g->graph);
        g->exec = nullptr;
        g->graph = nullptr;
    }
    if (!g || !g->exec) {
        // warm-up, then capture
        sigma_eager(c, c->Xg.p, c->Yg.p, nvec, precision);
        ADC_HIP(hipStreamSynchronize(E.stream));
        std::map<int, std::pair<void*, size_t>> used;
        const bool tune = E.autotune;
        E.autotune = false;          // shapes are tuned by now; no timing inside the capture
        E.scratch.touched = &used;
        hipGraph_t graph = nullptr;
        ADC_HIP(hipStreamBeginCapture(E.stream, hipStreamCaptureModeThreadLocal));
        try {
            sigma_eager(c, c->Xg.p, c->Yg.p, nvec, precision);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(E.stream, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            E.autotune = tune;
            E.scratch.touched = nullptr;
            throw;
        }
        ADC_HIP(hipStreamEndCapture(E.stream, &graph));
        E.autotune = tune;
        E.scratch.touched = nullptr;
        // the warm-up sized every buffer: nothing may have moved in the capture
        std::map<int, std::pair<void*, size_t>> before = used;
        ADC_REQUIRE(E.scratch.still_valid(before), "sigma graph: scratch moved during capture");
        hipGraphExec_t exec = nullptr;
        ADC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        if (!g) {
            c->graphs.emplace_back();
            g = &c->graphs.back();
        }
        ++c->graph_captures;
        g->nvec = nvec;
        g->precision = precision;
        g->slots = used;
        g->graph = graph;
        g->exec = exec;
    }
    ADC_HIP(hipGraphLaunch(g->exec, E.stream));
    ++c->graph_launches;
    ADC_HIP(hipMemcpyAsync(Y, c->Yg.p, bytes, hipMemcpyDeviceToDevice, E.stream));
    if (own) {
        // later null-stream work (and its synchronisations) wait for the replay
        ADC_HIP(hipEventRecord(c->gdone, c->gstream));
        ADC_HIP(hipStreamWaitEvent(nullptr, c->gdone, 0));
    }
}

hipGraph_t sigma_graph_ready(adc_ctx* c, int nvec, int precision) {
    if (nvec > 64 || !c->Xg.p || c->Xg.n < (size_t)nvec * c->dim) return nullptr;
    for (auto& g : c->graphs)
        if (g.nvec == nvec && g.precision == precision && g.exec &&
            c->E.scratch.still_valid(g.slots))
            return g.graph;
    return nullptr;
}

void sigma(adc_ctx* c, const double* X, double* Y, int nvec, int precision) {
    // process in chunks to bound the scratch footprint
    const int chunk = 64;
    for (int z0 = 0; z0 < nvec; z0 += chunk) {
        int nz = nvec - z0 < chunk ? nvec - z0 : chunk;
        const double* Xz = X + (long long)z0 * c->dim;
        double* Yz = Y + (long long)z0 * c->dim;
        if (c->use_graph && !c->E.timing && !c->E.ctr_log)
            sigma_graph(c, Xz, Yz, nz, precision);
        else
            sigma_eager(c, Xz, Yz, nz, precision);
    }
}

// Algorithmic flops of one sigma call (2 per multiply-add) for the contraction
// sequence above; pp is the particle-particle (EA) / hole-hole (IP) term, whose
// four-index rebuild is counted once per unique (ac|bd), Naux V^2 (V^2 + 1).
void sigma_cost(const adc_ctx* c, int nvec, double* total, double* pp) {
    if (c->uhf) {
        sigma_cost_uhf(c, nvec, total);
        *pp = 0.0;
        return;
    }
    const double n = nvec, O = c->O, V = c->V, Q = c->Q;
    double t = 0.0, p = 0.0;
    if (c->kind == ADC_EA) {
        t = n * (2 * V * V + 6 * O * V * V * Q + 4 * V * V * Q);
        if (c->order == 3) {
            t += n * (14 * O * O * V * V * V + 8 * O * V * V * Q + 2 * V * V * Q +
                      4 * O * O * O * V * V + 6 * O * O * O * V + 4 * O * V * Q + 6 * O * V * V);
            p = 2 * n * O * V * V * V * V + Q * V * V * (V * V + 1);
        }
    } else {
        t = n * (2 * O * O + 6 * O * O * V * Q + 4 * O * O * Q);
        if (c->order == 3) {
            t += n * (18 * O * O * O * V * V + 14 * O * O * O * V + 6 * O * O * V);
            p = 2 * n * V * O * O * O * O;
        }
    }
    *total = t + p;
    *pp = p;
}

template void sigma_block<double, double>(adc_ctx*, const double*, double*, int);
template void sigma_block<float, bf16_t>(adc_ctx*, const double*, double*, int);
template void sigma_block<float, float>(adc_ctx*, const double*, double*, int);

}  // namespace adc
