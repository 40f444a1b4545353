// Unrestricted (open-shell) EA/IP-ADC(2): the paper's UADC code path (Sec. II;
// the open-shell calculations of Sec. V.B) on the same contraction engine as
// the spin-adapted one, with alpha and beta blocks of the density-fitting
// factors (Eq. 38 for each pair of spins) instead of spin adaptation.
//
// Letters of the contraction strings: lower case alpha, upper case beta;
// i..o / I..L occupied, a..h, p / A..D, P virtual, Q auxiliary, z vectors.
//
// Resident tensors (FP64):
//   B blocks per spin, auxiliary index fastest: oo [i][j][Q], ov [i][a][Q],
//   vv [a][b][Q] (kept for EA; IP frees it once the singles are made);
//   first-order doubles  taa[i][j][a][b] = <ij||ab> / D, tbb likewise,
//                        tab[i][J][a][B] = (ia|JB) / D (alpha i, a; beta J, B);
//   Z^s[i][a][Q] = sum_jb t^ss_ijab B^Q_jb + sum over the other spin's (J, B)
//   of the mixed amplitudes (the one intermediate of the second-order 1p-1p /
//   1h-1h block and of the second-order singles);
//   M11 per spin, second-order singles t1 per spin, rho per spin (the
//   second-order part of the 1p/1h spectroscopic amplitudes).
//
// Vector layout (both spin sectors in one vector; see include/adc.h):
//   EA: Y1a [Va], Y1b [Vb], aaa [Oa][a<b], bab [Ob][Va][Vb], aab [Oa][Va][Vb],
//       bbb [Ob][A<B];
//   IP: Y1a [Oa], Y1b [Ob], aaa [Va][i<j], bab [Vb][Oa][Ob], aab [Va][Oa][Ob],
//       bbb [Vb][I<J].
// Packed pairs p < q row-major; a packed block is expanded to the full
// antisymmetric square before the contractions and packed back after.
//
// Working equations (second order; EA, the IP ones with the roles of the
// spaces exchanged and K = -M_-):
//   sigma1_a = M11 Y1 - sum_Q,b B^Q_ab W^Q_b,
//     W^Q_b (alpha) = sum_ic B^Q_ic Yaaa_ibc + sum_IC B^Q_IC Ybab_IbC,
//     W^Q_B (beta)  = sum_IC B^Q_IC Ybbb_IBC - sum_ib B^Q_ib Yaab_ibB;
//   sigma2 from U^Q_b = sum_a B^Q_ba Y1_a:
//     aaa_ibc = -(T_ibc - T_icb) + (e_b + e_c - e_i) Y,  T_ibc = sum_Q B^Q_ic U^Q_b,
//     bab_IbC = -sum_Q U^Q_b B^Q_IC + (...) Y,   aab_ibC = sum_Q B^Q_ib U^Q_C + (...) Y,
//     bbb like aaa;
// the spin-orbital derivation (from the definitions, Eqs. 7-10) and the
// reduction to these blocks are checked against the CPU oracle, whose
// spin-orbital equations are themselves checked against a Fock-space
// evaluation of Eqs. 7-14.
#include "context.hpp"

#include <algorithm>

namespace adc {

namespace {

unsigned nblk(long long n, int bs) {
    long long g = (n + bs - 1) / bs;
    if (g > (1LL << 22)) g = 1LL << 22;
    return (unsigned)(g < 1 ? 1 : g);
}

// scratch slots of this file
enum {
    U_Y1A = 200, U_Y1B, U_YAAA, U_YBAB, U_YAAB, U_YBBB, U_WA, U_WB, U_UA, U_UB, U_T, U_S1A, U_S1B,
    U_SMIX, U_TMP, U_XP
};

double* slotd(Engine& E, int s, size_t n) {
    return static_cast<double*>(E.scratch.get(s, std::max<size_t>(n, 1) * sizeof(double)));
}

// t[i][j][a][b] /= (e1_i + e2_j - e3_a - e4_b)
__global__ void k_denom_u(double* __restrict__ t, const double* __restrict__ e1,
                          const double* __restrict__ e2, const double* __restrict__ e3,
                          const double* __restrict__ e4, int n1, int n2, int n3, int n4) {
    const long long total = (long long)n1 * n2 * n3 * n4;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (long long)gridDim.x * blockDim.x) {
        long long r = x;
        const int b = (int)(r % n4); r /= n4;
        const int a = (int)(r % n3); r /= n3;
        const int j = (int)(r % n2);
        const int i = (int)(r / n2);
        t[x] /= e1[i] + e2[j] - e3[a] - e4[b];
    }
}

// x[r][p][q] <- x[r][p][q] - x[r][q][p] (one thread per pair p <= q of a row)
__global__ void k_antisym(double* __restrict__ x, long long rows, int n) {
    const long long nn = (long long)n * n;
    const long long total = rows * nn;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long r = e / nn, pq = e - r * nn;
        const int p = (int)(pq / n), q = (int)(pq - (long long)p * n);
        if (p > q) continue;
        double* xr = x + r * nn;
        if (p == q) {
            xr[pq] = 0.0;
            continue;
        }
        const double u = xr[(long long)p * n + q], v = xr[(long long)q * n + p];
        xr[(long long)p * n + q] = u - v;
        xr[(long long)q * n + p] = v - u;
    }
}

__device__ __forceinline__ long long pair_index(int p, int q, int n) {
    // p < q, row-major over p then q > p
    return (long long)p * n - (long long)p * (p + 1) / 2 + (q - p - 1);
}

// full[z][x][p][q] (contiguous) from packed[z*ld + off + x*P + k(p,q)], antisymmetric
__global__ void k_unpack(const double* __restrict__ in, long long ld, long long off,
                         double* __restrict__ out, int nvec, long long nx, int n) {
    const long long P = (long long)n * (n - 1) / 2;
    const long long nn = (long long)n * n;
    const long long total = (long long)nvec * nx * nn;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long zx = e / nn, pq = e - zx * nn;
        const long long z = zx / nx, x = zx - z * nx;
        const int p = (int)(pq / n), q = (int)(pq - (long long)p * n);
        const double* src = in + z * ld + off + x * P;
        double v = 0.0;
        if (p < q)
            v = src[pair_index(p, q, n)];
        else if (p > q)
            v = -src[pair_index(q, p, n)];
        out[e] = v;
    }
}

// out[z*ldo + off + x*P + k(p,q)] = s (T[z][x][p][q] - T[z][x][q][p])
//                                 + (sx ex[x] + sp (ep[p] + ep[q])) Y[z*ldy + off + x*P + k]
__global__ void k_pack(const double* __restrict__ T, const double* __restrict__ Y, long long ldy,
                       double* __restrict__ out, long long ldo, long long off, int nvec,
                       long long nx, int n, double s, const double* __restrict__ ex, double sx,
                       const double* __restrict__ ep, double sp) {
    const long long P = (long long)n * (n - 1) / 2;
    const long long nn = (long long)n * n;
    const long long total = (long long)nvec * nx * nn;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long zx = e / nn, pq = e - zx * nn;
        const int p = (int)(pq / n), q = (int)(pq - (long long)p * n);
        if (p >= q) continue;
        const long long z = zx / nx, x = zx - z * nx;
        const long long k = off + x * P + pair_index(p, q, n);
        const double* Tz = T + zx * nn;
        const double d = sx * ex[x] + sp * (ep[p] + ep[q]);
        out[z * ldo + k] = s * (Tz[(long long)p * n + q] - Tz[(long long)q * n + p]) + d * Y[z * ldy + k];
    }
}

// out[z*ldo + off + r] = S[z][r] + (sx ex[x] + sp (ep[p] + eq[q])) Y[z*ldy + off + r],
// r = (x, p, q) over [nx][np][nq]
__global__ void k_mixed(const double* __restrict__ S, const double* __restrict__ Y, long long ldy,
                        double* __restrict__ out, long long ldo, long long off, int nvec,
                        long long nx, int np, int nq, const double* __restrict__ ex, double sx,
                        const double* __restrict__ ep, const double* __restrict__ eq, double sp) {
    const long long len = nx * np * nq;
    const long long total = (long long)nvec * len;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long z = e / len, r = e - z * len;
        const long long x = r / ((long long)np * nq);
        const long long pq = r - x * np * nq;
        const int p = (int)(pq / nq), q = (int)(pq - (long long)p * nq);
        const double d = sx * ex[x] + sp * (ep[p] + eq[q]);
        out[z * ldo + off + r] = S[e] + d * Y[z * ldy + off + r];
    }
}

// diagonal of a packed block: d[off + x*P + k(p,q)] = sx ex[x] + sp (ep[p] + ep[q])
__global__ void k_diag_packed(double* __restrict__ d, long long off, long long nx, int n,
                              const double* __restrict__ ex, double sx,
                              const double* __restrict__ ep, double sp) {
    const long long nn = (long long)n * n;
    const long long P = (long long)n * (n - 1) / 2;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nx * nn;
         e += (long long)gridDim.x * blockDim.x) {
        const long long x = e / nn, pq = e - x * nn;
        const int p = (int)(pq / n), q = (int)(pq - (long long)p * n);
        if (p >= q) continue;
        d[off + x * P + pair_index(p, q, n)] = sx * ex[x] + sp * (ep[p] + ep[q]);
    }
}

__global__ void k_diag_mixed(double* __restrict__ d, long long off, long long nx, int np, int nq,
                             const double* __restrict__ ex, double sx,
                             const double* __restrict__ ep, const double* __restrict__ eq,
                             double sp) {
    const long long len = nx * np * nq;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < len;
         r += (long long)gridDim.x * blockDim.x) {
        const long long x = r / ((long long)np * nq);
        const long long pq = r - x * np * nq;
        const int p = (int)(pq / nq), q = (int)(pq - (long long)p * nq);
        d[off + r] = sx * ex[x] + sp * (ep[p] + eq[q]);
    }
}

// out[i][a] = s * in[i][a] / (e_i - e_a)  (second-order singles)
__global__ void k_denom1_u(double* __restrict__ t, const double* __restrict__ eo,
                           const double* __restrict__ ev, int O, int V) {
    const long long total = (long long)O * V;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(x / V), a = (int)(x - (long long)i * V);
        t[x] /= eo[i] - ev[a];
    }
}

void set_letters(adc_ctx* c, int nvec) {
    auto& u = c->uh;
    Engine& E = c->E;
    E.ext.O = u.Oa;
    E.ext.V = u.Va;
    E.ext.Q = c->Q;
    E.ext.Z = nvec;
    for (char ch : {'I', 'J', 'K', 'L'}) E.ext.extra[ch] = u.Ob;
    for (char ch : {'A', 'B', 'C', 'D', 'P'}) E.ext.extra[ch] = u.Vb;
    E.ext.extra['p'] = u.Va;
}

void to_device(adc_ctx* c, DBuf<double>& dst, const double* src, size_t n) {
    dst.alloc(n, &c->arena);
    ADC_HIP(hipMemcpyAsync(dst.p, src, n * sizeof(double), hipMemcpyDefault, c->E.stream));
}

}  // namespace

// ---------------------------------------------------------------------------
// setup: blocks, amplitudes, M11 per spin, diagonal
// ---------------------------------------------------------------------------
void setup_uhf(adc_ctx* c, const double* eps_a, const double* eps_b, const double* B_a,
               const double* B_b) {
    auto& u = c->uh;
    Engine& E = c->E;
    const int Oa = u.Oa, Ob = u.Ob, Va = u.Va, Vb = u.Vb, N = c->N, Q = c->Q;
    const bool ea = c->kind == ADC_EA;
    set_letters(c, 1);
    // inputs in device memory (host inputs are copied whole: the unrestricted
    // path is meant for systems whose B fits beside its copy)
    DBuf<double> hostB[2], epsd[2];
    const double* Bs[2] = {B_a, B_b};
    const double* es[2] = {eps_a, eps_b};
    for (int s = 0; s < 2; ++s) {
        hipPointerAttribute_t at;
        bool dev = hipPointerGetAttributes(&at, Bs[s]) == hipSuccess && at.type == hipMemoryTypeDevice;
        if (!dev) {
            (void)hipGetLastError();
            to_device(c, hostB[s], Bs[s], (size_t)Q * N * N);
            Bs[s] = hostB[s].p;
        }
        to_device(c, epsd[s], es[s], (size_t)N);
    }
    const int O[2] = {Oa, Ob}, V[2] = {Va, Vb};
    DBuf<double>* eo[2] = {&u.eoa, &u.eob};
    DBuf<double>* ev[2] = {&u.eva, &u.evb};
    DBuf<double>* Boo[2] = {&u.Booa, &u.Boob};
    DBuf<double>* Bov[2] = {&u.Bova, &u.Bovb};
    DBuf<double>* Bvv[2] = {&u.Bvva, &u.Bvvb};
    for (int s = 0; s < 2; ++s) {
        eo[s]->alloc(O[s], &c->arena);
        ev[s]->alloc(V[s], &c->arena);
        ADC_HIP(hipMemcpyAsync(eo[s]->p, epsd[s].p, O[s] * sizeof(double),
                               hipMemcpyDeviceToDevice, E.stream));
        ADC_HIP(hipMemcpyAsync(ev[s]->p, epsd[s].p + O[s], V[s] * sizeof(double),
                               hipMemcpyDeviceToDevice, E.stream));
        Boo[s]->alloc((size_t)O[s] * O[s] * Q, &c->arena);
        Bov[s]->alloc((size_t)O[s] * V[s] * Q, &c->arena);
        stage_block(E, Bs[s], Q, N, 0, O[s], 0, O[s], Boo[s]->p);
        stage_block(E, Bs[s], Q, N, 0, O[s], O[s], V[s], Bov[s]->p);
        // the vv block: the EA sigma, and the second-order singles of both
        // kinds (released after setup for IP)
        Bvv[s]->alloc((size_t)V[s] * V[s] * Q, &c->arena);
        stage_block(E, Bs[s], Q, N, O[s], V[s], O[s], V[s], Bvv[s]->p);
    }
    ADC_HIP(hipStreamSynchronize(E.stream));
    for (int s = 0; s < 2; ++s) hostB[s].release();
    c->phase("unrestricted: DF factors staged");

    // first-order doubles
    u.taa.alloc((size_t)Oa * Oa * Va * Va, &c->arena);
    u.tbb.alloc((size_t)Ob * Ob * Vb * Vb, &c->arena);
    u.tab.alloc((size_t)Oa * Ob * Va * Vb, &c->arena);
    ctr<double>(E, 1.0, "iaQ", u.Bova.p, "jbQ", u.Bova.p, 0.0, "ijab", u.taa.p);
    ctr<double>(E, 1.0, "IAQ", u.Bovb.p, "JBQ", u.Bovb.p, 0.0, "IJAB", u.tbb.p);
    ctr<double>(E, 1.0, "iaQ", u.Bova.p, "JBQ", u.Bovb.p, 0.0, "iJaB", u.tab.p);
    hipLaunchKernelGGL(k_antisym, dim3(nblk((long long)Oa * Oa * Va * Va, 256)), dim3(256), 0,
                       E.stream, u.taa.p, (long long)Oa * Oa, Va);
    hipLaunchKernelGGL(k_antisym, dim3(nblk((long long)Ob * Ob * Vb * Vb, 256)), dim3(256), 0,
                       E.stream, u.tbb.p, (long long)Ob * Ob, Vb);
    hipLaunchKernelGGL(k_denom_u, dim3(nblk((long long)Oa * Oa * Va * Va, 256)), dim3(256), 0,
                       E.stream, u.taa.p, u.eoa.p, u.eoa.p, u.eva.p, u.eva.p, Oa, Oa, Va, Va);
    hipLaunchKernelGGL(k_denom_u, dim3(nblk((long long)Ob * Ob * Vb * Vb, 256)), dim3(256), 0,
                       E.stream, u.tbb.p, u.eob.p, u.eob.p, u.evb.p, u.evb.p, Ob, Ob, Vb, Vb);
    hipLaunchKernelGGL(k_denom_u, dim3(nblk((long long)Oa * Ob * Va * Vb, 256)), dim3(256), 0,
                       E.stream, u.tab.p, u.eoa.p, u.eob.p, u.eva.p, u.evb.p, Oa, Ob, Va, Vb);
    ADC_HIP(hipGetLastError());
    c->phase("unrestricted: first-order doubles");

    // Z^s[i][a][Q]
    DBuf<double> Za, Zb;
    Za.alloc((size_t)Oa * Va * Q, &c->arena);
    Zb.alloc((size_t)Ob * Vb * Q, &c->arena);
    ctr<double>(E, 1.0, "ijab", u.taa.p, "jbQ", u.Bova.p, 0.0, "iaQ", Za.p);
    ctr<double>(E, 1.0, "iJaB", u.tab.p, "JBQ", u.Bovb.p, 1.0, "iaQ", Za.p);
    ctr<double>(E, 1.0, "IJAB", u.tbb.p, "JBQ", u.Bovb.p, 0.0, "IAQ", Zb.p);
    ctr<double>(E, 1.0, "jIbA", u.tab.p, "jbQ", u.Bova.p, 1.0, "IAQ", Zb.p);

    // second-order singles: t1[i][a] = (-sum B^Q_ab Z_ibQ + sum B^Q_ji Z_jaQ) / (e_i - e_a)
    u.t1a.alloc((size_t)Oa * Va, &c->arena);
    u.t1b.alloc((size_t)Ob * Vb, &c->arena);
    ctr<double>(E, -1.0, "abQ", u.Bvva.p, "ibQ", Za.p, 0.0, "ia", u.t1a.p);
    ctr<double>(E, -1.0, "ABQ", u.Bvvb.p, "IBQ", Zb.p, 0.0, "IA", u.t1b.p);
    if (!ea) {
        ADC_HIP(hipStreamSynchronize(E.stream));
        u.Bvva.release();
        u.Bvvb.release();
    }
    ctr<double>(E, 1.0, "jiQ", u.Booa.p, "jaQ", Za.p, 1.0, "ia", u.t1a.p);
    ctr<double>(E, 1.0, "JIQ", u.Boob.p, "JAQ", Zb.p, 1.0, "IA", u.t1b.p);
    hipLaunchKernelGGL(k_denom1_u, dim3(nblk((long long)Oa * Va, 256)), dim3(256), 0, E.stream,
                       u.t1a.p, u.eoa.p, u.eva.p, Oa, Va);
    hipLaunchKernelGGL(k_denom1_u, dim3(nblk((long long)Ob * Vb, 256)), dim3(256), 0, E.stream,
                       u.t1b.p, u.eob.p, u.evb.p, Ob, Vb);
    ADC_HIP(hipGetLastError());

    // M11 per spin: sgn diag(e) - 1/2 (tau + tau^T)
    const int n1a = ea ? Va : Oa, n1b = ea ? Vb : Ob;
    u.M11a.alloc((size_t)n1a * n1a, &c->arena);
    u.M11b.alloc((size_t)n1b * n1b, &c->arena);
    DBuf<double> tau;
    tau.alloc((size_t)std::max(n1a * n1a, n1b * n1b), &c->arena);
    if (ea) {
        ctr<double>(E, 1.0, "kaQ", Za.p, "kbQ", u.Bova.p, 0.0, "ab", tau.p);
        symmetrize_m11(E, u.M11a.p, tau.p, u.eva.p, Va, 1.0);
        ctr<double>(E, 1.0, "KAQ", Zb.p, "KBQ", u.Bovb.p, 0.0, "AB", tau.p);
        symmetrize_m11(E, u.M11b.p, tau.p, u.evb.p, Vb, 1.0);
    } else {
        ctr<double>(E, 1.0, "icQ", Za.p, "jcQ", u.Bova.p, 0.0, "ij", tau.p);
        symmetrize_m11(E, u.M11a.p, tau.p, u.eoa.p, Oa, -1.0);
        ctr<double>(E, 1.0, "ICQ", Zb.p, "JCQ", u.Bovb.p, 0.0, "IJ", tau.p);
        symmetrize_m11(E, u.M11b.p, tau.p, u.eob.p, Ob, -1.0);
    }
    // rho per spin (second-order part of the 1p / 1h spectroscopic amplitudes)
    u.rhoa.alloc((size_t)n1a * n1a, &c->arena);
    u.rhob.alloc((size_t)n1b * n1b, &c->arena);
    if (ea) {
        ctr<double>(E, 1.0, "klac", u.taa.p, "klbc", u.taa.p, 0.0, "ab", u.rhoa.p);
        ctr<double>(E, 2.0, "kLaC", u.tab.p, "kLbC", u.tab.p, 1.0, "ab", u.rhoa.p);
        ctr<double>(E, 1.0, "KLAC", u.tbb.p, "KLBC", u.tbb.p, 0.0, "AB", u.rhob.p);
        ctr<double>(E, 2.0, "kLcA", u.tab.p, "kLcB", u.tab.p, 1.0, "AB", u.rhob.p);
    } else {
        ctr<double>(E, 1.0, "ikcd", u.taa.p, "jkcd", u.taa.p, 0.0, "ij", u.rhoa.p);
        ctr<double>(E, 2.0, "iKcD", u.tab.p, "jKcD", u.tab.p, 1.0, "ij", u.rhoa.p);
        ctr<double>(E, 1.0, "IKCD", u.tbb.p, "JKCD", u.tbb.p, 0.0, "IJ", u.rhob.p);
        ctr<double>(E, 2.0, "kIcD", u.tab.p, "kJcD", u.tab.p, 1.0, "IJ", u.rhob.p);
    }
    c->phase("unrestricted: second-order singles, 1p-1p / 1h-1h block, rho");

    // diagonal: M11 diagonals, zeroth order of the four 2p1h / 2h1p blocks
    c->diag.alloc((size_t)c->dim, &c->arena);
    set_diag(E, c->diag.p, u.M11a.p, n1a);
    set_diag(E, c->diag.p + n1a, u.M11b.p, n1b);
    const long long* off = u.off;
    if (ea) {
        hipLaunchKernelGGL(k_diag_packed, dim3(nblk((long long)Oa * Va * Va, 256)), dim3(256), 0,
                           E.stream, c->diag.p, off[2], (long long)Oa, Va, u.eoa.p, -1.0, u.eva.p, 1.0);
        hipLaunchKernelGGL(k_diag_mixed, dim3(nblk((long long)Ob * Va * Vb, 256)), dim3(256), 0,
                           E.stream, c->diag.p, off[3], (long long)Ob, Va, Vb, u.eob.p, -1.0,
                           u.eva.p, u.evb.p, 1.0);
        hipLaunchKernelGGL(k_diag_mixed, dim3(nblk((long long)Oa * Va * Vb, 256)), dim3(256), 0,
                           E.stream, c->diag.p, off[4], (long long)Oa, Va, Vb, u.eoa.p, -1.0,
                           u.eva.p, u.evb.p, 1.0);
        hipLaunchKernelGGL(k_diag_packed, dim3(nblk((long long)Ob * Vb * Vb, 256)), dim3(256), 0,
                           E.stream, c->diag.p, off[5], (long long)Ob, Vb, u.eob.p, -1.0, u.evb.p, 1.0);
    } else {
        hipLaunchKernelGGL(k_diag_packed, dim3(nblk((long long)Va * Oa * Oa, 256)), dim3(256), 0,
                           E.stream, c->diag.p, off[2], (long long)Va, Oa, u.eva.p, 1.0, u.eoa.p, -1.0);
        hipLaunchKernelGGL(k_diag_mixed, dim3(nblk((long long)Vb * Oa * Ob, 256)), dim3(256), 0,
                           E.stream, c->diag.p, off[3], (long long)Vb, Oa, Ob, u.evb.p, 1.0,
                           u.eoa.p, u.eob.p, -1.0);
        hipLaunchKernelGGL(k_diag_mixed, dim3(nblk((long long)Va * Oa * Ob, 256)), dim3(256), 0,
                           E.stream, c->diag.p, off[4], (long long)Va, Oa, Ob, u.eva.p, 1.0,
                           u.eoa.p, u.eob.p, -1.0);
        hipLaunchKernelGGL(k_diag_packed, dim3(nblk((long long)Vb * Ob * Ob, 256)), dim3(256), 0,
                           E.stream, c->diag.p, off[5], (long long)Vb, Ob, u.evb.p, 1.0, u.eob.p, -1.0);
    }
    ADC_HIP(hipGetLastError());
    ADC_HIP(hipStreamSynchronize(E.stream));
    E.scratch.clear();
    c->phase("unrestricted: setup done");
}

// ---------------------------------------------------------------------------
// sigma (FP64 at every precision level)
// ---------------------------------------------------------------------------
namespace {

// the four 2p1h / 2h1p blocks of X as contiguous tensors (packed ones expanded)
struct UBlocks {
    double *Y1a, *Y1b, *Yaaa, *Ybab, *Yaab, *Ybbb;
};

UBlocks load_blocks(adc_ctx* c, const double* X, int nvec) {
    auto& u = c->uh;
    Engine& E = c->E;
    const long long dim = c->dim;
    const bool ea = c->kind == ADC_EA;
    const long long* off = u.off;
    const int n1a = (int)(off[1] - off[0]), n1b = (int)(off[2] - off[1]);
    // extents (x, p) of the packed blocks: EA [O][V][V], IP [V][O][O]
    const long long xa = ea ? u.Oa : u.Va, xb = ea ? u.Ob : u.Vb;
    const int pa = ea ? u.Va : u.Oa, pb = ea ? u.Vb : u.Ob;
    const long long lbab = off[4] - off[3], laab = off[5] - off[4];
    UBlocks b;
    b.Y1a = slotd(E, U_Y1A, (size_t)nvec * n1a);
    b.Y1b = slotd(E, U_Y1B, (size_t)nvec * n1b);
    b.Yaaa = slotd(E, U_YAAA, (size_t)nvec * xa * pa * pa);
    b.Ybab = slotd(E, U_YBAB, (size_t)nvec * lbab);
    b.Yaab = slotd(E, U_YAAB, (size_t)nvec * laab);
    b.Ybbb = slotd(E, U_YBBB, (size_t)nvec * xb * pb * pb);
    copy_rows<double, double>(E, X, dim, off[0], b.Y1a, n1a, 0, nvec, n1a, 0.0);
    copy_rows<double, double>(E, X, dim, off[1], b.Y1b, n1b, 0, nvec, n1b, 0.0);
    copy_rows<double, double>(E, X, dim, off[3], b.Ybab, lbab, 0, nvec, lbab, 0.0);
    copy_rows<double, double>(E, X, dim, off[4], b.Yaab, laab, 0, nvec, laab, 0.0);
    hipLaunchKernelGGL(k_unpack, dim3(nblk((long long)nvec * xa * pa * pa, 256)), dim3(256), 0,
                       E.stream, X, dim, off[2], b.Yaaa, nvec, xa, pa);
    hipLaunchKernelGGL(k_unpack, dim3(nblk((long long)nvec * xb * pb * pb, 256)), dim3(256), 0,
                       E.stream, X, dim, off[5], b.Ybbb, nvec, xb, pb);
    ADC_HIP(hipGetLastError());
    return b;
}

}  // namespace

void sigma_uhf(adc_ctx* c, const double* X, double* Yout, int nvec) {
    auto& u = c->uh;
    Engine& E = c->E;
    set_letters(c, nvec);
    const int Oa = u.Oa, Ob = u.Ob, Va = u.Va, Vb = u.Vb, Q = c->Q;
    const long long dim = c->dim;
    const bool ea = c->kind == ADC_EA;
    const long long* off = u.off;
    UBlocks b = load_blocks(c, X, nvec);
    double* S1a = slotd(E, U_S1A, (size_t)nvec * (off[1] - off[0]));
    double* S1b = slotd(E, U_S1B, (size_t)nvec * (off[2] - off[1]));
    if (ea) {
        double* Wa = slotd(E, U_WA, (size_t)nvec * Va * Q);
        double* Wb = slotd(E, U_WB, (size_t)nvec * Vb * Q);
        ctr<double>(E, 1.0, "icQ", u.Bova.p, "zibc", b.Yaaa, 0.0, "zbQ", Wa);
        ctr<double>(E, 1.0, "ICQ", u.Bovb.p, "zIbC", b.Ybab, 1.0, "zbQ", Wa);
        ctr<double>(E, 1.0, "ICQ", u.Bovb.p, "zIBC", b.Ybbb, 0.0, "zBQ", Wb);
        ctr<double>(E, -1.0, "ibQ", u.Bova.p, "zibB", b.Yaab, 1.0, "zBQ", Wb);
        ctr<double>(E, 1.0, "ab", u.M11a.p, "zb", b.Y1a, 0.0, "za", S1a);
        ctr<double>(E, -1.0, "abQ", u.Bvva.p, "zbQ", Wa, 1.0, "za", S1a);
        ctr<double>(E, 1.0, "AB", u.M11b.p, "zB", b.Y1b, 0.0, "zA", S1b);
        ctr<double>(E, -1.0, "ABQ", u.Bvvb.p, "zBQ", Wb, 1.0, "zA", S1b);
        // sigma2 from U^Q_b = sum_a B^Q_ba Y1_a
        double* Ua = slotd(E, U_UA, (size_t)nvec * Va * Q);
        double* Ub = slotd(E, U_UB, (size_t)nvec * Vb * Q);
        ctr<double>(E, 1.0, "baQ", u.Bvva.p, "za", b.Y1a, 0.0, "zbQ", Ua);
        ctr<double>(E, 1.0, "BAQ", u.Bvvb.p, "zA", b.Y1b, 0.0, "zBQ", Ub);
        double* T = slotd(E, U_T, (size_t)nvec * std::max((long long)Oa * Va * Va,
                                                          (long long)Ob * Vb * Vb));
        ctr<double>(E, 1.0, "icQ", u.Bova.p, "zbQ", Ua, 0.0, "zibc", T);
        hipLaunchKernelGGL(k_pack, dim3(nblk((long long)nvec * Oa * Va * Va, 256)), dim3(256), 0,
                           E.stream, T, X, dim, Yout, dim, off[2], nvec, (long long)Oa, Va, -1.0,
                           u.eoa.p, -1.0, u.eva.p, 1.0);
        ctr<double>(E, 1.0, "ICQ", u.Bovb.p, "zBQ", Ub, 0.0, "zIBC", T);
        hipLaunchKernelGGL(k_pack, dim3(nblk((long long)nvec * Ob * Vb * Vb, 256)), dim3(256), 0,
                           E.stream, T, X, dim, Yout, dim, off[5], nvec, (long long)Ob, Vb, -1.0,
                           u.eob.p, -1.0, u.evb.p, 1.0);
        double* Sm = slotd(E, U_SMIX, (size_t)nvec * std::max(off[4] - off[3], off[5] - off[4]));
        ctr<double>(E, -1.0, "zbQ", Ua, "ICQ", u.Bovb.p, 0.0, "zIbC", Sm);
        hipLaunchKernelGGL(k_mixed, dim3(nblk((long long)nvec * Ob * Va * Vb, 256)), dim3(256), 0,
                           E.stream, Sm, X, dim, Yout, dim, off[3], nvec, (long long)Ob, Va, Vb,
                           u.eob.p, -1.0, u.eva.p, u.evb.p, 1.0);
        ctr<double>(E, 1.0, "ibQ", u.Bova.p, "zCQ", Ub, 0.0, "zibC", Sm);
        hipLaunchKernelGGL(k_mixed, dim3(nblk((long long)nvec * Oa * Va * Vb, 256)), dim3(256), 0,
                           E.stream, Sm, X, dim, Yout, dim, off[4], nvec, (long long)Oa, Va, Vb,
                           u.eoa.p, -1.0, u.eva.p, u.evb.p, 1.0);
    } else {
        double* Wa = slotd(E, U_WA, (size_t)nvec * Oa * Q);
        double* Wb = slotd(E, U_WB, (size_t)nvec * Ob * Q);
        ctr<double>(E, 1.0, "kaQ", u.Bova.p, "zajk", b.Yaaa, 0.0, "zjQ", Wa);
        ctr<double>(E, 1.0, "KAQ", u.Bovb.p, "zAjK", b.Ybab, 1.0, "zjQ", Wa);
        ctr<double>(E, 1.0, "JAQ", u.Bovb.p, "zAKJ", b.Ybbb, 0.0, "zKQ", Wb);
        ctr<double>(E, -1.0, "jaQ", u.Bova.p, "zajK", b.Yaab, 1.0, "zKQ", Wb);
        ctr<double>(E, 1.0, "ij", u.M11a.p, "zj", b.Y1a, 0.0, "zi", S1a);
        ctr<double>(E, -1.0, "ijQ", u.Booa.p, "zjQ", Wa, 1.0, "zi", S1a);
        ctr<double>(E, 1.0, "IJ", u.M11b.p, "zJ", b.Y1b, 0.0, "zI", S1b);
        ctr<double>(E, -1.0, "IJQ", u.Boob.p, "zJQ", Wb, 1.0, "zI", S1b);
        double* Ua = slotd(E, U_UA, (size_t)nvec * Oa * Q);
        double* Ub = slotd(E, U_UB, (size_t)nvec * Ob * Q);
        ctr<double>(E, 1.0, "jiQ", u.Booa.p, "zi", b.Y1a, 0.0, "zjQ", Ua);
        ctr<double>(E, 1.0, "JIQ", u.Boob.p, "zI", b.Y1b, 0.0, "zJQ", Ub);
        double* T = slotd(E, U_T, (size_t)nvec * std::max((long long)Va * Oa * Oa,
                                                          (long long)Vb * Ob * Ob));
        ctr<double>(E, 1.0, "zjQ", Ua, "kaQ", u.Bova.p, 0.0, "zajk", T);
        hipLaunchKernelGGL(k_pack, dim3(nblk((long long)nvec * Va * Oa * Oa, 256)), dim3(256), 0,
                           E.stream, T, X, dim, Yout, dim, off[2], nvec, (long long)Va, Oa, -1.0,
                           u.eva.p, 1.0, u.eoa.p, -1.0);
        ctr<double>(E, 1.0, "zJQ", Ub, "KAQ", u.Bovb.p, 0.0, "zAJK", T);
        hipLaunchKernelGGL(k_pack, dim3(nblk((long long)nvec * Vb * Ob * Ob, 256)), dim3(256), 0,
                           E.stream, T, X, dim, Yout, dim, off[5], nvec, (long long)Vb, Ob, -1.0,
                           u.evb.p, 1.0, u.eob.p, -1.0);
        double* Sm = slotd(E, U_SMIX, (size_t)nvec * std::max(off[4] - off[3], off[5] - off[4]));
        ctr<double>(E, -1.0, "zjQ", Ua, "KAQ", u.Bovb.p, 0.0, "zAjK", Sm);
        hipLaunchKernelGGL(k_mixed, dim3(nblk((long long)nvec * Vb * Oa * Ob, 256)), dim3(256), 0,
                           E.stream, Sm, X, dim, Yout, dim, off[3], nvec, (long long)Vb, Oa, Ob,
                           u.evb.p, 1.0, u.eoa.p, u.eob.p, -1.0);
        ctr<double>(E, 1.0, "jaQ", u.Bova.p, "zKQ", Ub, 0.0, "zajK", Sm);
        hipLaunchKernelGGL(k_mixed, dim3(nblk((long long)nvec * Va * Oa * Ob, 256)), dim3(256), 0,
                           E.stream, Sm, X, dim, Yout, dim, off[4], nvec, (long long)Va, Oa, Ob,
                           u.eva.p, 1.0, u.eoa.p, u.eob.p, -1.0);
    }
    ADC_HIP(hipGetLastError());
    copy_rows<double, double>(E, S1a, off[1] - off[0], 0, Yout, dim, off[0], nvec,
                              off[1] - off[0], 0.0);
    copy_rows<double, double>(E, S1b, off[2] - off[1], 0, Yout, dim, off[1], nvec,
                              off[2] - off[1], 0.0);
}

// ---------------------------------------------------------------------------
// spectroscopic amplitudes X [nvec][2N]: alpha orbitals 0..N-1, then beta
// ---------------------------------------------------------------------------
void spec_amplitudes_uhf(adc_ctx* c, const double* vecs, int nvec, double* Xout) {
    auto& u = c->uh;
    Engine& E = c->E;
    set_letters(c, nvec);
    const int Oa = u.Oa, Ob = u.Ob, Va = u.Va, Vb = u.Vb, N = c->N;
    const bool ea = c->kind == ADC_EA;
    UBlocks b = load_blocks(c, vecs, nvec);
    double* Xp = slotd(E, U_XP, (size_t)nvec * std::max(std::max(Oa, Ob), std::max(Va, Vb)));
    const long long ld = 2LL * N;
    auto put = [&](long long col0, int n) {
        copy_rows<double, double>(E, Xp, n, 0, Xout, ld, col0, nvec, n, 0.0);
    };
    if (ea) {
        // X_a = Y1_a - 1/4 rho Y1
        copy_rows<double, double>(E, b.Y1a, Va, 0, Xp, Va, 0, nvec, Va, 0.0);
        ctr<double>(E, -0.25, "ab", u.rhoa.p, "zb", b.Y1a, 1.0, "za", Xp);
        put(Oa, Va);
        copy_rows<double, double>(E, b.Y1b, Vb, 0, Xp, Vb, 0, nvec, Vb, 0.0);
        ctr<double>(E, -0.25, "AB", u.rhob.p, "zB", b.Y1b, 1.0, "zA", Xp);
        put(N + Ob, Vb);
        // X_k (occupied) = t1 Y1 - 1/2 t Yss + / - tab Ymixed
        ctr<double>(E, 1.0, "ka", u.t1a.p, "za", b.Y1a, 0.0, "zk", Xp);
        ctr<double>(E, -0.5, "ikab", u.taa.p, "ziab", b.Yaaa, 1.0, "zk", Xp);
        ctr<double>(E, 1.0, "kIaB", u.tab.p, "zIaB", b.Ybab, 1.0, "zk", Xp);
        put(0, Oa);
        ctr<double>(E, 1.0, "KA", u.t1b.p, "zA", b.Y1b, 0.0, "zK", Xp);
        ctr<double>(E, -0.5, "IKAB", u.tbb.p, "zIAB", b.Ybbb, 1.0, "zK", Xp);
        ctr<double>(E, -1.0, "iKaB", u.tab.p, "ziaB", b.Yaab, 1.0, "zK", Xp);
        put(N, Ob);
    } else {
        copy_rows<double, double>(E, b.Y1a, Oa, 0, Xp, Oa, 0, nvec, Oa, 0.0);
        ctr<double>(E, -0.25, "ij", u.rhoa.p, "zj", b.Y1a, 1.0, "zi", Xp);
        put(0, Oa);
        copy_rows<double, double>(E, b.Y1b, Ob, 0, Xp, Ob, 0, nvec, Ob, 0.0);
        ctr<double>(E, -0.25, "IJ", u.rhob.p, "zJ", b.Y1b, 1.0, "zI", Xp);
        put(N, Ob);
        // X_p (virtual) = -t1^T Y1 - 1/2 t Yss + / - tab Ymixed
        ctr<double>(E, -1.0, "ip", u.t1a.p, "zi", b.Y1a, 0.0, "zp", Xp);
        ctr<double>(E, -0.5, "jkap", u.taa.p, "zajk", b.Yaaa, 1.0, "zp", Xp);
        ctr<double>(E, 1.0, "jKpA", u.tab.p, "zAjK", b.Ybab, 1.0, "zp", Xp);
        put(Oa, Va);
        ctr<double>(E, -1.0, "IP", u.t1b.p, "zI", b.Y1b, 0.0, "zP", Xp);
        ctr<double>(E, -0.5, "JKAP", u.tbb.p, "zAJK", b.Ybbb, 1.0, "zP", Xp);
        ctr<double>(E, -1.0, "jKaP", u.tab.p, "zajK", b.Yaab, 1.0, "zP", Xp);
        put(N + Ob, Vb);
    }
}

void sigma_cost_uhf(const adc_ctx* c, int nvec, double* total) {
    const auto& u = c->uh;
    const double n = nvec, Q = c->Q, Oa = u.Oa, Ob = u.Ob, Va = u.Va, Vb = u.Vb;
    double t;
    if (c->kind == ADC_EA)
        t = 2 * (Va * Va + Vb * Vb) + 4 * Q * (Oa * Va * Va + Ob * Va * Vb + Oa * Va * Vb + Ob * Vb * Vb) +
            4 * Q * (Va * Va + Vb * Vb);
    else
        t = 2 * (Oa * Oa + Ob * Ob) + 4 * Q * (Va * Oa * Oa + Vb * Oa * Ob + Va * Oa * Ob + Vb * Ob * Ob) +
            4 * Q * (Oa * Oa + Ob * Ob);
    *total = n * t;
}

}  // namespace adc
