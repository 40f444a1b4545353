// The 1p-1p (EA) / 1h-1h (IP) block applied to the trial vectors on the fly
// (the alternative to step 3 of Sec. III.A the paper describes: instead of
// precomputing M11, its contribution sum_b M_ab Y_b is recomputed every
// iteration through intermediates made from Y, so no O^2 V^4 block build is
// needed and each term costs at most O^3 V^2 (or V^2 Naux) per vector).
//
// Every term below is a term of the precomputed block (setup.hip, setup3.hip)
// with the sum over the block's second index taken first:
//   sum_b M_ab Y_b  and  sum_b M_ba Y_b  for the symmetrised pieces.
// Always FP64 (the block is a small part of sigma and sets the 1p / 1h rows).
#include "context.hpp"

namespace adc {

namespace {

// scratch slots, one per live range (a slot is regrown only after its last reader)
enum FlySlot { F_A = 80, F_B, F_C, F_D, F_E, F_T, F_V = 90, F_BV, F_G, F_H, F_N, F_HO };

double* fs(Engine& E, int slot, size_t n) { return (double*)E.scratch.get(slot, n * sizeof(double)); }

// out[z][p] = sg e[p] Y[z][p]  (the zeroth-order block)
__global__ void k_diag_rows(const double* __restrict__ e, const double* __restrict__ Y,
                            double* __restrict__ out, long long n1, long long total, double sg) {
    for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < total;
         o += (long long)gridDim.x * blockDim.x)
        out[o] = sg * e[o % n1] * Y[o];
}

void zeroth(Engine& E, const double* e, const double* Y, double* out, long long n1, long long nvec,
            double sg) {
    const long long total = n1 * nvec;
    hipLaunchKernelGGL(k_diag_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, E.stream,
                       e, Y, out, n1, total, sg);
    ADC_HIP(hipGetLastError());
}

// EA: out[z][a] = sum_b M_ab Y1[z][b]
void fly_ea(adc_ctx* c, const double* Y, double* out, int nvec) {
    Engine& E = c->E;
    const size_t Z = nvec, O = c->O, V = c->V, Q = c->Q;
    const size_t OOV = O * O * V, OVV = O * V * V, VQ = V * Q;
    const double *t = c->t.p, *ovov = c->ovov.p;
    double* acc = fs(E, F_T, Z * V);   // the -1/2 (tau + tau^T) and other sums
    double* W = fs(E, F_A, Z * OOV);
    double* X = fs(E, F_B, Z * OOV);
    zeroth(E, c->ev.p, Y, out, V, Z, 1.0);   // zeroth order
    // second (and, with u, third) order: -1/2 (tau + tau^T), tau_ab = x_jk^ca [2 (jc|kb) - (jb|kc)]
    auto tau = [&](const double* x) {
        ctr<double>(E, 2.0, "jckb", ovov, "zb", Y, 0.0, "zjck", W);
        ctr<double>(E, -1.0, "jbkc", ovov, "zb", Y, 1.0, "zjck", W);
        ctr<double>(E, 1.0, "jkca", x, "zjck", W, 0.0, "za", acc);
        ctr<double>(E, 1.0, "jkcb", x, "zb", Y, 0.0, "zjkc", X);
        ctr<double>(E, 2.0, "zjkc", X, "jcka", ovov, 1.0, "za", acc);
        ctr<double>(E, -1.0, "zjkc", X, "jakc", ovov, 1.0, "za", acc);
        axpy<double>(E, -0.5, acc, out, Z * V);
    };
    tau(t);
    if (c->order < 3) return;
    const double *tt = c->tt.p, *u = c->u.p, *Du = c->Du.p, *Lam = c->Lam.p, *oovv = c->oovv.p,
                 *oooo = c->oooo.p, *Bov = c->Bov.p, *Bvv = c->Bvv.p, *s = c->s.p;
    tau(u);
    // s terms: 4 (jc|ab) s_jc - (T + T^T), T_ab = sum_cQ (ac|Q) Ys[b][c][Q],
    // Ys[b][c][Q] = sum_j (jb|Q) s_jc
    {
        double* v = fs(E, F_V, Q);
        double* Bv = fs(E, F_BV, V * V);
        ctr<double>(E, 1.0, "jc", s, "jcQ", Bov, 0.0, "Q", v);
        ctr<double>(E, 1.0, "abQ", Bvv, "Q", v, 0.0, "ab", Bv);
        ctr<double>(E, 4.0, "ab", Bv, "zb", Y, 1.0, "za", out);
        double* G = fs(E, F_G, Z * O * Q);
        double* H = fs(E, F_H, Z * VQ);
        ctr<double>(E, 1.0, "jbQ", Bov, "zb", Y, 0.0, "zjQ", G);
        ctr<double>(E, 1.0, "jc", s, "zjQ", G, 0.0, "zcQ", H);
        ctr<double>(E, -1.0, "acQ", Bvv, "zcQ", H, 1.0, "za", out);
        ctr<double>(E, 1.0, "bcQ", Bvv, "zb", Y, 0.0, "zcQ", H);     // K[z][c][Q]
        ctr<double>(E, 1.0, "jc", s, "zcQ", H, 0.0, "zjQ", G);
        ctr<double>(E, -1.0, "jaQ", Bov, "zjQ", G, 1.0, "za", out);
        // Pt terms: 2 Pt.(ce|ab) and - Zp(ac|Q) (bc|Q), Zp[a][c][Q] = Pt_ce (ae|Q)
        ctr<double>(E, 1.0, "abQ", Bvv, "Q", c->wq.p, 0.0, "ab", Bv);
        ctr<double>(E, 2.0, "ab", Bv, "zb", Y, 1.0, "za", out);
        double* N = fs(E, F_N, Z * VQ);
        ctr<double>(E, 1.0, "ce", c->Pt.p, "zcQ", H, 0.0, "zeQ", N);
        ctr<double>(E, -1.0, "aeQ", Bvv, "zeQ", N, 1.0, "za", out);
    }
    // -1/2 (pi + pi^T), pi_ae = t~_jk^ba Du_jk^be
    ctr<double>(E, 1.0, "jkbe", Du, "ze", Y, 0.0, "zjkb", W);
    ctr<double>(E, 1.0, "jkba", tt, "zjkb", W, 0.0, "za", acc);
    ctr<double>(E, 1.0, "jkbe", tt, "ze", Y, 0.0, "zjkb", W);
    ctr<double>(E, 1.0, "jkba", Du, "zjkb", W, 1.0, "za", acc);
    axpy<double>(E, -0.5, acc, out, Z * V);
    // W = t_jk^cb Y_b, W2 = t_jk^bc Y_b, Wt = t~_jk^cb Y_b   ([z][j][k][c])
    double* W2 = fs(E, F_C, Z * OOV);
    double* Wt = fs(E, F_D, Z * OOV);
    ctr<double>(E, 1.0, "jkcb", t, "zb", Y, 0.0, "zjkc", W);
    ctr<double>(E, 1.0, "jkbc", t, "zb", Y, 0.0, "zjkc", W2);
    ctr<double>(E, 1.0, "jkcb", tt, "zb", Y, 0.0, "zjkc", Wt);
    double* U = fs(E, F_E, Z * OOV);
    // hole-hole ladder: + t_jk^cb Zo_jk^ca - 2 t_jk^cb Zo_kj^ca, Zo_kj^ca = (mk|lj) t_lm^ca
    ctr<double>(E, 1.0, "mjlk", oooo, "zjkc", W, 0.0, "zlmc", U);
    ctr<double>(E, 1.0, "lmca", t, "zlmc", U, 1.0, "za", out);
    ctr<double>(E, 1.0, "mklj", oooo, "zjkc", W, 0.0, "zlmc", U);
    ctr<double>(E, -2.0, "lmca", t, "zlmc", U, 1.0, "za", out);
    // rings, R1[j][c][k][a] = t~_lj^dc (ld|ka), R2 = t~_lj^dc (lk|ad), R3 = t~_lj^cd (lk|ad):
    //   - t~_jk^cb R1_jcka + t_jk^cb R2_jcka + t_jk^bc R3_jcka
    ctr<double>(E, 1.0, "zjkc", Wt, "ljdc", tt, 0.0, "zkld", U);
    ctr<double>(E, -1.0, "zkld", U, "ldka", ovov, 1.0, "za", out);
    ctr<double>(E, 1.0, "zjkc", W, "ljdc", tt, 0.0, "zkld", U);
    ctr<double>(E, 1.0, "zkld", U, "lkad", oovv, 1.0, "za", out);
    ctr<double>(E, 1.0, "zjkc", W2, "ljcd", tt, 0.0, "zkld", U);
    ctr<double>(E, 1.0, "zkld", U, "lkad", oovv, 1.0, "za", out);
    //   + t_jk^cb (R3 + R1)[j][a][k][c] + t_jk^bc (R2 - 2 R1)[j][a][k][c]
    ctr<double>(E, 1.0, "zjkc", W, "ldkc", ovov, 0.0, "zjld", U);
    ctr<double>(E, 1.0, "ljda", tt, "zjld", U, 1.0, "za", out);
    ctr<double>(E, 1.0, "zjkc", W, "lkcd", oovv, 0.0, "zjld", U);
    ctr<double>(E, 1.0, "ljad", tt, "zjld", U, 1.0, "za", out);
    ctr<double>(E, 1.0, "zjkc", W2, "lkcd", oovv, 0.0, "zjld", U);
    ctr<double>(E, -2.0, "zjkc", W2, "ldkc", ovov, 1.0, "zjld", U);
    ctr<double>(E, 1.0, "ljda", tt, "zjld", U, 1.0, "za", out);
    // Lambda terms: - t_jk^cb Lambda~_jk^ca - t_jk^ac Lambda~_jk^bc (Lambda~ = 2 Lambda - Lambda^(ab))
    ctr<double>(E, -2.0, "zjkc", W, "jkca", Lam, 1.0, "za", out);
    ctr<double>(E, 1.0, "zjkc", W, "jkac", Lam, 1.0, "za", out);
    ctr<double>(E, 1.0, "jkbc", Lam, "zb", Y, 0.0, "zjkc", U);
    ctr<double>(E, -2.0, "jkac", t, "zjkc", U, 1.0, "za", out);
    ctr<double>(E, 1.0, "jkcb", Lam, "zb", Y, 0.0, "zjkc", U);
    ctr<double>(E, 1.0, "jkac", t, "zjkc", U, 1.0, "za", out);
    // P terms: + P_kl (lb|ka) - 2 P_kl (lk|ab)
    ctr<double>(E, 1.0, "lbka", ovov, "zb", Y, 0.0, "zlka", U);
    ctr<double>(E, 1.0, "kl", c->P.p, "zlka", U, 1.0, "za", out);
    ctr<double>(E, 1.0, "lkab", oovv, "zb", Y, 0.0, "zlka", U);
    ctr<double>(E, -2.0, "kl", c->P.p, "zlka", U, 1.0, "za", out);
    // Q5 (lk|cb) - Q6 (lb|kc), Q5 = t~_jk^cd t_lj^da + t~_jk^dc t_lj^ad, Q6 = t~_jk^dc t~_lj^ad
    double* U2 = fs(E, F_V, Z * OVV);
    ctr<double>(E, 1.0, "lkcb", oovv, "zb", Y, 0.0, "zlkc", U);
    ctr<double>(E, 1.0, "jkcd", tt, "zlkc", U, 0.0, "zjdl", U2);
    ctr<double>(E, 1.0, "ljda", t, "zjdl", U2, 1.0, "za", out);
    ctr<double>(E, 1.0, "jkdc", tt, "zlkc", U, 0.0, "zjdl", U2);
    ctr<double>(E, 1.0, "ljad", t, "zjdl", U2, 1.0, "za", out);
    ctr<double>(E, 1.0, "lbkc", ovov, "zb", Y, 0.0, "zlkc", U);
    ctr<double>(E, 1.0, "jkdc", tt, "zlkc", U, 0.0, "zjdl", U2);
    ctr<double>(E, -1.0, "ljad", tt, "zjdl", U2, 1.0, "za", out);
}

// IP: out[z][i] = sum_j M_ij Y1[z][j]
void fly_ip(adc_ctx* c, const double* Y, double* out, int nvec) {
    Engine& E = c->E;
    const size_t Z = nvec, O = c->O, V = c->V;
    const size_t OVV = O * V * V, OO = O * O;
    const double *t = c->t.p, *ovov = c->ovov.p;
    double* acc = fs(E, F_T, Z * O);
    double* W = fs(E, F_A, Z * OVV);
    double* X = fs(E, F_B, Z * OVV);
    zeroth(E, c->eo.p, Y, out, O, Z, -1.0);   // zeroth order
    // -1/2 (kappa + kappa^T), kappa_ij = x_ik^bc [2 (jb|kc) - (jc|kb)]
    auto kappa = [&](const double* x) {
        ctr<double>(E, 2.0, "jbkc", ovov, "zj", Y, 0.0, "zbkc", W);
        ctr<double>(E, -1.0, "jckb", ovov, "zj", Y, 1.0, "zbkc", W);
        ctr<double>(E, 1.0, "ikbc", x, "zbkc", W, 0.0, "zi", acc);
        ctr<double>(E, 1.0, "jkbc", x, "zj", Y, 0.0, "zkbc", X);
        ctr<double>(E, 2.0, "zkbc", X, "ibkc", ovov, 1.0, "zi", acc);
        ctr<double>(E, -1.0, "zkbc", X, "ickb", ovov, 1.0, "zi", acc);
        axpy<double>(E, -0.5, acc, out, Z * O);
    };
    kappa(t);
    if (c->order < 3) return;
    const double *tt = c->tt.p, *u = c->u.p, *Du = c->Du.p, *Lam = c->Lam.p, *oovv = c->oovv.p,
                 *oooo = c->oooo.p, *ooov = c->ooov.p, *s = c->s.p;
    kappa(u);
    // the O x O pieces (s terms, hole-hole pieces, Pt terms), made per call and applied
    {
        double* H = fs(E, F_HO, OO);
        ctr<double>(E, -4.0, "kb", s, "jikb", ooov, 0.0, "ij", H);
        ctr<double>(E, 1.0, "kb", s, "kijb", ooov, 1.0, "ij", H);
        ctr<double>(E, 1.0, "kb", s, "jkib", ooov, 1.0, "ij", H);
        ctr<double>(E, -2.0, "jklm", c->P7.p, "milk", oooo, 1.0, "ij", H);
        ctr<double>(E, 1.0, "jklm", c->P7.p, "mkli", oooo, 1.0, "ij", H);
        ctr<double>(E, -2.0, "iklm", c->P7.p, "jmkl", oooo, 1.0, "ij", H);
        ctr<double>(E, 1.0, "iklm", c->P7.p, "jlkm", oooo, 1.0, "ij", H);
        ctr<double>(E, 2.0, "lm", c->P.p, "jiml", oooo, 1.0, "ij", H);
        ctr<double>(E, -1.0, "lm", c->P.p, "jlmi", oooo, 1.0, "ij", H);
        ctr<double>(E, 1.0, "bd", c->Pt.p, "jdib", ovov, 1.0, "ij", H);
        ctr<double>(E, -2.0, "bd", c->Pt.p, "jibd", oovv, 1.0, "ij", H);
        ctr<double>(E, 1.0, "ij", H, "zj", Y, 1.0, "zi", out);
    }
    // -1/2 (pi + pi^T), pi_ij = t~_ik^bc Du_jk^bc
    ctr<double>(E, 1.0, "jkbc", Du, "zj", Y, 0.0, "zkbc", W);
    ctr<double>(E, 1.0, "ikbc", tt, "zkbc", W, 0.0, "zi", acc);
    ctr<double>(E, 1.0, "jkbc", tt, "zj", Y, 0.0, "zkbc", W);
    ctr<double>(E, 1.0, "ikbc", Du, "zkbc", W, 1.0, "zi", acc);
    axpy<double>(E, -0.5, acc, out, Z * O);
    // rings, R1[j][c][k][a] = t~_lj^dc (ld|ka), R2 = t~_lj^dc (lk|ad), R3 = t~_lj^cd (lk|ad),
    // Ra = R2 - 2 R1, Rb = R3 + R1:
    //   t_jk^bc Ra_kcib + t_jk^bc Rb_kbic + t_ik^bc Ra_jbkc + t_ik^bc Rb_jckb
    double* U = fs(E, F_C, Z * OVV);
    double* G = fs(E, F_D, Z * OVV);
    ctr<double>(E, 1.0, "jkbc", t, "zj", Y, 0.0, "zkbc", W);          // V1
    ctr<double>(E, 1.0, "zkbc", W, "lkdc", tt, 0.0, "zlbd", U);
    ctr<double>(E, 1.0, "zlbd", U, "libd", oovv, 1.0, "zi", out);
    ctr<double>(E, -2.0, "zlbd", U, "ldib", ovov, 1.0, "zi", out);
    ctr<double>(E, 1.0, "zkbc", W, "lkbd", tt, 0.0, "zlcd", U);
    ctr<double>(E, 1.0, "zlcd", U, "licd", oovv, 1.0, "zi", out);
    ctr<double>(E, 1.0, "zkbc", W, "lkdb", tt, 0.0, "zlcd", U);
    ctr<double>(E, 1.0, "zlcd", U, "ldic", ovov, 1.0, "zi", out);
    ctr<double>(E, 1.0, "ljdb", tt, "zj", Y, 0.0, "zldb", U);          // A1
    ctr<double>(E, 1.0, "zldb", U, "lkcd", oovv, 0.0, "zbkc", G);
    ctr<double>(E, -2.0, "zldb", U, "ldkc", ovov, 1.0, "zbkc", G);
    ctr<double>(E, 1.0, "ikbc", t, "zbkc", G, 1.0, "zi", out);
    ctr<double>(E, 1.0, "ljcd", tt, "zj", Y, 0.0, "zlcd", U);          // A2
    ctr<double>(E, 1.0, "zlcd", U, "lkbd", oovv, 0.0, "zckb", G);
    ctr<double>(E, 1.0, "ljdc", tt, "zj", Y, 0.0, "zldc", U);          // A3
    ctr<double>(E, 1.0, "zldc", U, "ldkb", ovov, 1.0, "zckb", G);
    ctr<double>(E, 1.0, "ikbc", t, "zckb", G, 1.0, "zi", out);
    // Q7 (jl|dc) + Q8 (jc|ld) + Q9 [(jl|db) - 2 (jb|ld)], Q7[i][c][l][d] = t_ik^bc t~_kl^db,
    // Q8 = t_ik^bc t~_kl^bd, Q9[i][b][l][d] = t_ik^bc t~_kl^cd
    ctr<double>(E, 1.0, "jldc", oovv, "zj", Y, 0.0, "zldc", U);
    ctr<double>(E, 1.0, "kldb", tt, "zldc", U, 0.0, "zkbc", G);
    ctr<double>(E, 1.0, "ikbc", t, "zkbc", G, 1.0, "zi", out);
    ctr<double>(E, 1.0, "jcld", ovov, "zj", Y, 0.0, "zcld", U);
    ctr<double>(E, 1.0, "klbd", tt, "zcld", U, 0.0, "zkbc", G);
    ctr<double>(E, 1.0, "ikbc", t, "zkbc", G, 1.0, "zi", out);
    ctr<double>(E, 1.0, "jldb", oovv, "zj", Y, 0.0, "zldb", U);
    ctr<double>(E, 1.0, "klcd", tt, "zldb", U, 0.0, "zkcb", G);
    ctr<double>(E, 1.0, "jbld", ovov, "zj", Y, 0.0, "zbld", U);
    ctr<double>(E, -2.0, "klcd", tt, "zbld", U, 1.0, "zkcb", G);
    ctr<double>(E, 1.0, "ikbc", t, "zkcb", G, 1.0, "zi", out);
    // Lambda term: - t_ik^bc Lambda~_jk^bc
    ctr<double>(E, 1.0, "jkbc", Lam, "zj", Y, 0.0, "zkbc", U);
    ctr<double>(E, -2.0, "ikbc", t, "zkbc", U, 1.0, "zi", out);
    ctr<double>(E, 1.0, "jkcb", Lam, "zj", Y, 0.0, "zkbc", U);
    ctr<double>(E, 1.0, "ikbc", t, "zkbc", U, 1.0, "zi", out);
}

}  // namespace

void m11_fly(adc_ctx* c, const double* Y1, double* S1, int nvec) {
    Engine& E = c->E;
    const long long zold = E.ext.Z;
    E.ext.Z = nvec;
    if (c->kind == ADC_EA)
        fly_ea(c, Y1, S1, nvec);
    else
        fly_ip(c, Y1, S1, nvec);
    E.ext.Z = zold;
}

}  // namespace adc
