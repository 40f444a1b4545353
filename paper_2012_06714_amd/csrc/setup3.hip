// Third-order additions to the setup: second-order doubles u through the
// particle-particle ladder Lambda (rebuilt from B like the sigma vvvv term),
// third-order singles w, the third-order 1p-1p (EA) or 1h-1h (IP) block and the
// intermediates of the second-order coupling (Gamma; for IP also the
// precontracted Omega and Pi blocks) and of the transition moments.
//
// Notation: t~ = 2 t_ij^ab - t_ij^ba (same for u~, Lambda~); (pq|rs) from the
// resident blocks or as sum_Q B B; every contraction is a ctr() call whose
// einsum string names the indices.  All of it runs once, in FP64.
#include "context.hpp"

#include <algorithm>

namespace adc {


namespace {
struct Buf {
    DBuf<double> b;
    double* get(adc_ctx* c, size_t n) {
        b.alloc(n, &c->arena);
        return b.p;
    }
};
void tilde_of(adc_ctx* c, const double* x, double* out) {
    Engine& E = c->E;
    permute<double>(E, -1.0, "ijab", x, 0.0, "ijba", out);
    axpy<double>(E, 2.0, x, out, (size_t)c->O * c->O * c->V * c->V);
}
}  // namespace

// third-order terms of the 1p-1p block (EA); M holds the second-order block on entry
static void m11_third_ea(adc_ctx* c, double* M, const double* t, const double* tt,
                         const double* u, const double* Du, const double* Lt, const double* P,
                         const double* R1, const double* R2, const double* R3, const double* wq,
                         const double* Zp) {
    Engine& E = c->E;
    const int O = c->O, V = c->V, Q = c->Q;
    const size_t OO = (size_t)O * O, VV = (size_t)V * V;
    const double *Bov = c->Bov.p, *Bvv = c->Bvv.p, *ovov = c->ovov.p, *oovv = c->oovv.p,
                 *oooo = c->oooo.p;
    Buf Tb, Wb;
    double* T = Tb.get(c, VV);
    double* v = Wb.get(c, (size_t)Q);
    // -1/2 (tau[u] + tau[u]^T), tau_ab = u_jk^ca [2 (jc|kb) - (jb|kc)]
    ctr<double>(E, 2.0, "jkca", u, "jckb", ovov, 0.0, "ab", T);
    ctr<double>(E, -1.0, "jkca", u, "jbkc", ovov, 1.0, "ab", T);
    permute<double>(E, -0.5, "ab", T, 1.0, "ab", M);
    permute<double>(E, -0.5, "ba", T, 1.0, "ab", M);
    // s terms: 4 (jc|ab) s_jc - (jb|ac) s_jc - (ja|bc) s_jc
    ctr<double>(E, 1.0, "jc", c->s.p, "jcQ", Bov, 0.0, "Q", v);
    ctr<double>(E, 4.0, "abQ", Bvv, "Q", v, 1.0, "ab", M);
    {
        Buf Ysb;
        double* Ys = Ysb.get(c, VV * Q);
        ctr<double>(E, 1.0, "jbQ", Bov, "jc", c->s.p, 0.0, "bcQ", Ys);
        ctr<double>(E, 1.0, "acQ", Bvv, "bcQ", Ys, 0.0, "ab", T);
    }
    permute<double>(E, -1.0, "ab", T, 1.0, "ab", M);
    permute<double>(E, -1.0, "ba", T, 1.0, "ab", M);
    // -1/2 (pi + pi^T), pi_ae = t~_jk^ba Du_jk^be
    ctr<double>(E, 1.0, "jkba", tt, "jkbe", Du, 0.0, "ae", T);
    permute<double>(E, -0.5, "ab", T, 1.0, "ab", M);
    permute<double>(E, -0.5, "ba", T, 1.0, "ab", M);
    // hole-hole ladder: Zo_kj^ca = (mk|lj) t_lm^ca
    Buf Zb, Xb;
    double* Zo = Zb.get(c, OO * VV);
    ctr<double>(E, 1.0, "mklj", oooo, "lmca", t, 0.0, "kjca", Zo);
    ctr<double>(E, 1.0, "jkcb", t, "jkca", Zo, 1.0, "ab", M);
    ctr<double>(E, -2.0, "jkcb", t, "kjca", Zo, 1.0, "ab", M);
    // rings
    double* Rx = Xb.get(c, OO * VV);
    ctr<double>(E, -1.0, "jkcb", tt, "jcka", R1, 1.0, "ab", M);
    ctr<double>(E, 1.0, "jkcb", t, "jcka", R2, 1.0, "ab", M);
    ctr<double>(E, 1.0, "jkbc", t, "jcka", R3, 1.0, "ab", M);
    ADC_HIP(hipMemcpyAsync(Rx, R3, OO * VV * sizeof(double), hipMemcpyDeviceToDevice, E.stream));
    axpy<double>(E, 1.0, R1, Rx, OO * VV);
    ctr<double>(E, 1.0, "jkcb", t, "jakc", Rx, 1.0, "ab", M);
    ADC_HIP(hipMemcpyAsync(Rx, R2, OO * VV * sizeof(double), hipMemcpyDeviceToDevice, E.stream));
    axpy<double>(E, -2.0, R1, Rx, OO * VV);
    ctr<double>(E, 1.0, "jkbc", t, "jakc", Rx, 1.0, "ab", M);
    ctr<double>(E, 1.0, "kl", P, "lbka", ovov, 1.0, "ab", M);
    ctr<double>(E, -2.0, "kl", P, "lkab", oovv, 1.0, "ab", M);
    // Q5 = t~_jk^cd t_lj^da + t~_jk^dc t_lj^ad ; Q6 = t~_jk^dc t~_lj^ad   ([k][c][l][a])
    ctr<double>(E, 1.0, "jkcd", tt, "ljda", t, 0.0, "kcla", Zo);
    ctr<double>(E, 1.0, "jkdc", tt, "ljad", t, 1.0, "kcla", Zo);
    ctr<double>(E, 1.0, "jkdc", tt, "ljad", tt, 0.0, "kcla", Rx);
    ctr<double>(E, 1.0, "kcla", Zo, "lkcb", oovv, 1.0, "ab", M);
    ctr<double>(E, -1.0, "kcla", Rx, "lbkc", ovov, 1.0, "ab", M);
    // particle-particle terms through Lambda~
    ctr<double>(E, -1.0, "jkcb", t, "jkca", Lt, 1.0, "ab", M);
    ctr<double>(E, -1.0, "jkac", t, "jkbc", Lt, 1.0, "ab", M);
    // 2 Pt.(ce|ab) - Pt.(cb|ae)
    ctr<double>(E, 2.0, "abQ", Bvv, "Q", wq, 1.0, "ab", M);
    ctr<double>(E, -1.0, "acQ", Zp, "bcQ", Bvv, 1.0, "ab", M);
}

// third-order terms of the 1h-1h block (IP); M holds the second-order block on entry
static void m11_third_ip(adc_ctx* c, double* M, const double* t, const double* tt,
                         const double* u, const double* Du, const double* Lt, const double* P,
                         const double* P7, const double* Pt, const double* R1, const double* R2,
                         const double* R3) {
    Engine& E = c->E;
    const int O = c->O, V = c->V;
    const size_t OO = (size_t)O * O, VV = (size_t)V * V;
    const double *ooov = c->ooov.p, *ovov = c->ovov.p, *oovv = c->oovv.p, *oooo = c->oooo.p;
    Buf Tb, Xb, Yb, Zb;
    double* T = Tb.get(c, OO);
    // -1/2 (kappa[u] + kappa[u]^T), kappa_ij = u_ik^bc [2 (jb|kc) - (jc|kb)]
    ctr<double>(E, 2.0, "ikbc", u, "jbkc", ovov, 0.0, "ij", T);
    ctr<double>(E, -1.0, "ikbc", u, "jckb", ovov, 1.0, "ij", T);
    permute<double>(E, -0.5, "ij", T, 1.0, "ij", M);
    permute<double>(E, -0.5, "ji", T, 1.0, "ij", M);
    // s terms
    ctr<double>(E, -4.0, "kb", c->s.p, "jikb", ooov, 1.0, "ij", M);
    ctr<double>(E, 1.0, "kb", c->s.p, "kijb", ooov, 1.0, "ij", M);
    ctr<double>(E, 1.0, "kb", c->s.p, "jkib", ooov, 1.0, "ij", M);
    // -1/2 (pi + pi^T), pi_ij = t~_ik^bc Du_jk^bc
    ctr<double>(E, 1.0, "ikbc", tt, "jkbc", Du, 0.0, "ij", T);
    permute<double>(E, -0.5, "ij", T, 1.0, "ij", M);
    permute<double>(E, -0.5, "ji", T, 1.0, "ij", M);
    // hole-hole pieces
    ctr<double>(E, -2.0, "jklm", P7, "milk", oooo, 1.0, "ij", M);
    ctr<double>(E, 1.0, "jklm", P7, "mkli", oooo, 1.0, "ij", M);
    ctr<double>(E, -2.0, "iklm", P7, "jmkl", oooo, 1.0, "ij", M);
    ctr<double>(E, 1.0, "iklm", P7, "jlkm", oooo, 1.0, "ij", M);
    ctr<double>(E, 2.0, "lm", P, "jiml", oooo, 1.0, "ij", M);
    ctr<double>(E, -1.0, "lm", P, "jlmi", oooo, 1.0, "ij", M);
    // rings with (R2 - 2 R1) and (R3 + R1)
    double* Ra = Xb.get(c, OO * VV);
    double* Rb = Yb.get(c, OO * VV);
    ADC_HIP(hipMemcpyAsync(Ra, R2, OO * VV * sizeof(double), hipMemcpyDeviceToDevice, E.stream));
    axpy<double>(E, -2.0, R1, Ra, OO * VV);
    ADC_HIP(hipMemcpyAsync(Rb, R3, OO * VV * sizeof(double), hipMemcpyDeviceToDevice, E.stream));
    axpy<double>(E, 1.0, R1, Rb, OO * VV);
    ctr<double>(E, 1.0, "jkbc", t, "kcib", Ra, 1.0, "ij", M);
    ctr<double>(E, 1.0, "jkbc", t, "kbic", Rb, 1.0, "ij", M);
    ctr<double>(E, 1.0, "ikbc", t, "jbkc", Ra, 1.0, "ij", M);
    ctr<double>(E, 1.0, "ikbc", t, "jckb", Rb, 1.0, "ij", M);
    ctr<double>(E, 1.0, "bd", Pt, "jdib", ovov, 1.0, "ij", M);
    ctr<double>(E, -2.0, "bd", Pt, "jibd", oovv, 1.0, "ij", M);
    // Q7 = t_ik^bc t~_kl^db, Q8 = t_ik^bc t~_kl^bd ([i][c][l][d]); Q9 = t_ik^bc t~_kl^cd ([i][b][l][d])
    double* Qx = Zb.get(c, OO * VV);
    ctr<double>(E, 1.0, "ikbc", t, "kldb", tt, 0.0, "icld", Qx);
    ctr<double>(E, 1.0, "icld", Qx, "jldc", oovv, 1.0, "ij", M);
    ctr<double>(E, 1.0, "ikbc", t, "klbd", tt, 0.0, "icld", Qx);
    ctr<double>(E, 1.0, "icld", Qx, "jcld", ovov, 1.0, "ij", M);
    ctr<double>(E, 1.0, "ikbc", t, "klcd", tt, 0.0, "ibld", Qx);
    ctr<double>(E, 1.0, "ibld", Qx, "jldb", oovv, 1.0, "ij", M);
    ctr<double>(E, -2.0, "ibld", Qx, "jbld", ovov, 1.0, "ij", M);
    // particle-particle term through Lambda~
    ctr<double>(E, -1.0, "ikbc", t, "jkbc", Lt, 1.0, "ij", M);
}

void setup_adc3(adc_ctx* c, const double* tt, const double* X1) {
    const bool ea = c->kind == ADC_EA;
    Engine& E = c->E;
    const int O = c->O, V = c->V, Q = c->Q;
    const size_t OO = (size_t)O * O, VV = (size_t)V * V, OV = (size_t)O * V;
    const double* t = c->t.p;
    const double *Bov = c->Bov.p, *Bvv = c->Bvv.p, *Boo = c->Boo.p;
    const double *ovov = c->ovov.p, *ooov = c->ooov.p;

    c->oovv.alloc(OO * VV, &c->arena);
    ctr<double>(E, 1.0, "ijQ", Boo, "abQ", Bvv, 0.0, "ijab", c->oovv.p);
    c->oooo.alloc(OO * OO, &c->arena);
    ctr<double>(E, 1.0, "ijQ", Boo, "klQ", Boo, 0.0, "ijkl", c->oooo.p);
    const double *oovv = c->oovv.p, *oooo = c->oooo.p;

    // ---- Gamma_jb = G_bj + H_bj + Ds_jb -------------------------------------------
    //   G_bj = t_kl^cb [(jk|cl) - 2 (jl|ck)],  H_bj = t~_jk^cd [2 (dk|cb) - (db|ck)] = X1 . Bvv
    Buf Gb, Dsb;
    double* G = Gb.get(c, OV);
    ctr<double>(E, 1.0, "klcb", t, "jklc", ooov, 0.0, "jb", G);
    ctr<double>(E, -2.0, "klcb", t, "jlkc", ooov, 1.0, "jb", G);
    double* Ds = Dsb.get(c, OV);
    mul_denom1(E, c->s.p, Ds, c->eo.p, c->ev.p, O, V);
    c->gam.alloc(OV, &c->arena);
    ctr<double>(E, 1.0, "jcQ", X1, "cbQ", Bvv, 0.0, "jb", c->gam.p);
    axpy<double>(E, 1.0, G, c->gam.p, OV);
    axpy<double>(E, 1.0, Ds, c->gam.p, OV);

    // ---- particle-particle ladder and second-order doubles --------------------------
    Buf Lb, Ltb;
    double* Lam = Lb.get(c, OO * VV);
    // Lambda_ij^ab = (ac|bd) t_ij^cd; t_ij^cd = t_ji^dc, so the mirrored products are rows
    // of the direct ones
    vvvv_apply<double, double>(c, Bvv, t, Lam, (long long)OO, O);
    E.scratch.clear();   // the rebuilt slab and operand copies are not needed again here
    c->u.alloc(OO * VV, &c->arena);
    double* u = c->u.p;
    ctr<double>(E, 1.0, "klba", t, "likj", oooo, 0.0, "ijab", u);
    axpy<double>(E, 1.0, Lam, u, OO * VV);
    ctr<double>(E, -1.0, "jkca", t, "kibc", oovv, 1.0, "ijab", u);
    ctr<double>(E, -1.0, "jkbc", t, "kiac", oovv, 1.0, "ijab", u);
    ctr<double>(E, -1.0, "ikac", t, "kjbc", oovv, 1.0, "ijab", u);
    ctr<double>(E, -1.0, "ikcb", t, "kjac", oovv, 1.0, "ijab", u);
    ctr<double>(E, 1.0, "jkbc", tt, "kcia", ovov, 1.0, "ijab", u);
    ctr<double>(E, 1.0, "ikac", tt, "kcjb", ovov, 1.0, "ijab", u);
    divide_denom2(E, u, c->eo.p, c->ev.p, O, V, 1.0);              // u = R / (e_i+e_j-e_a-e_b)
    double* Lt = Ltb.get(c, OO * VV);
    tilde_of(c, Lam, Lt);
    Lb.b.release();
    Buf Dub, utb;
    double* Du = Dub.get(c, OO * VV);
    mul_denom2(E, u, Du, c->eo.p, c->ev.p, O, V);                  // (e_a+e_b-e_i-e_j) u
    double* ut = utb.get(c, OO * VV);
    tilde_of(c, u, ut);

    // ---- shared intermediates ----------------------------------------------------------
    Buf P_b, P7b, Ptb, wqb, Zpb;
    double* P = P_b.get(c, OO);              // P_kl = t_jk^cd t~_lj^dc
    ctr<double>(E, 1.0, "jkcd", t, "ljdc", tt, 0.0, "kl", P);
    double* P7 = P7b.get(c, OO * OO);        // P7_ijkl = t_ij^bc t_kl^cb
    ctr<double>(E, 1.0, "ijbc", t, "klcb", t, 0.0, "ijkl", P7);
    double* Pt = Ptb.get(c, VV);             // Pt_ce = t_jk^cd t~_kj^de
    ctr<double>(E, 1.0, "jkcd", t, "kjde", tt, 0.0, "ce", Pt);
    double* wq = wqb.get(c, (size_t)Q);      // sum_ce Pt_ce B^Q_ce
    ctr<double>(E, 1.0, "ce", Pt, "ceQ", Bvv, 0.0, "Q", wq);
    double* Zp = Zpb.get(c, VV * Q);         // Zp[a][c][Q] = Pt_ce B^Q_ae
    ctr<double>(E, 1.0, "aeQ", Bvv, "ce", Pt, 0.0, "acQ", Zp);

    // ---- third-order 1p-1p / 1h-1h block -------------------------------------------------
    {
        // ring intermediates R[j][c][k][a] = t~_lj^dc (ld|ka), t~_lj^dc (lk|ad), t~_lj^cd (lk|ad)
        Buf r1, r2, r3;
        double* R1 = r1.get(c, OO * VV);
        double* R2 = r2.get(c, OO * VV);
        double* R3 = r3.get(c, OO * VV);
        ctr<double>(E, 1.0, "ljdc", tt, "ldka", ovov, 0.0, "jcka", R1);
        ctr<double>(E, 1.0, "ljdc", tt, "lkad", oovv, 0.0, "jcka", R2);
        ctr<double>(E, 1.0, "ljcd", tt, "lkad", oovv, 0.0, "jcka", R3);
        if (ea)
            m11_third_ea(c, c->M11.p, t, tt, u, Du, Lt, P, R1, R2, R3, wq, Zp);
        else
            m11_third_ip(c, c->M11.p, t, tt, u, Du, Lt, P, P7, Pt, R1, R2, R3);
    }
    E.scratch.clear();
    Ltb.b.release();
    Dub.b.release();

    // ---- third-order singles w --------------------------------------------------------
    c->w.alloc(OV, &c->arena);
    double* R = c->w.p;
    ctr<double>(E, 1.0, "jkba", u, "jikb", ooov, 0.0, "ia", R);
    ctr<double>(E, -2.0, "jkba", u, "kijb", ooov, 1.0, "ia", R);
    ctr<double>(E, -1.0, "jb", c->s.p, "jiab", oovv, 1.0, "ia", R);
    ctr<double>(E, 3.0, "jb", c->s.p, "jbia", ovov, 1.0, "ia", R);
    ctr<double>(E, -0.5, "jb", c->s.p, "ibja", ovov, 1.0, "ia", R);
    {
        Buf x2b;
        double* X2 = x2b.get(c, OV * Q);
        ctr<double>(E, 1.0, "ijbc", ut, "jcQ", Bov, 0.0, "ibQ", X2);
        ctr<double>(E, 1.0, "ibQ", X2, "abQ", Bvv, 1.0, "ia", R);
        // t~ (Gamma - Ds/2)
        Buf gb;
        double* gmh = gb.get(c, OV);
        ADC_HIP(hipMemcpyAsync(gmh, c->gam.p, OV * sizeof(double), hipMemcpyDeviceToDevice,
                               E.stream));
        axpy<double>(E, -0.5, Ds, gmh, OV);
        ctr<double>(E, 1.0, "ijab", tt, "jb", gmh, 1.0, "ia", R);
        // P_kl [(li|ka) - 2 (lk|ia)]
        ctr<double>(E, 1.0, "kl", P, "lika", ooov, 1.0, "ia", R);
        ctr<double>(E, -2.0, "kl", P, "lkia", ooov, 1.0, "ia", R);
        // PA, PB ([k][b][l][a]), PC ([k][c][l][a])
        Buf pb;
        double* PX = pb.get(c, OO * VV);
        ctr<double>(E, 1.0, "jkbc", t, "ljac", tt, 0.0, "kbla", PX);
        ctr<double>(E, 1.0, "kbla", PX, "likb", ooov, 1.0, "ia", R);
        ctr<double>(E, 1.0, "jkbc", t, "ljca", tt, 0.0, "kbla", PX);
        ctr<double>(E, 1.0, "kbla", PX, "lkib", ooov, 1.0, "ia", R);
        ctr<double>(E, 1.0, "jkbc", t, "ljab", tt, 0.0, "kcla", PX);
        ctr<double>(E, 1.0, "kcla", PX, "lkic", ooov, 1.0, "ia", R);
        ctr<double>(E, -2.0, "kcla", PX, "likc", ooov, 1.0, "ia", R);
        // P7 [2 (jk|la) - (jl|ka)]
        ctr<double>(E, -1.0, "ijkl", P7, "jlka", ooov, 1.0, "ia", R);
        ctr<double>(E, 2.0, "ijkl", P7, "jkla", ooov, 1.0, "ia", R);
        // Pt terms: 2 Pt.(bd|ai) - Pt.(ib|ad)
        ctr<double>(E, 2.0, "Q", wq, "iaQ", Bov, 1.0, "ia", R);
        ctr<double>(E, -1.0, "ibQ", Bov, "abQ", Zp, 1.0, "ia", R);
        // t~ X1 Bvv
        ctr<double>(E, 1.0, "ijbc", tt, "jcQ", X1, 0.0, "ibQ", X2);
        ctr<double>(E, 1.0, "ibQ", X2, "abQ", Bvv, 1.0, "ia", R);
        // Pq[i][c][k][d] = t_ij^bc t~_jk^db + t_ij^cb t~_jk^bd ; -(dc|ak)
        ctr<double>(E, 1.0, "ijbc", t, "jkdb", tt, 0.0, "ickd", PX);
        ctr<double>(E, 1.0, "ijcb", t, "jkbd", tt, 1.0, "ickd", PX);
        Buf tqb;
        double* Tq = tqb.get(c, OO * Q);
        ctr<double>(E, 1.0, "ickd", PX, "cdQ", Bvv, 0.0, "ikQ", Tq);
        ctr<double>(E, -1.0, "ikQ", Tq, "kaQ", Bov, 1.0, "ia", R);
    }
    Zpb.b.release();
    {
        // slabs S_m[b][c][d] = (b m|c d), m in a block of occupied orbitals:
        //   w:  R_ma += sum_jkd [sum_bc t_jk^bc (S_m[c][b][d] - 2 S_m[b][c][d])] t_jk^ad
        //   IP: Omega[m][k][j][b] = t_kj^cd (S_m[c][d][b] - 2 S_m[d][c][b])
        //       Pi[m][j][i][a]    = t_ji^bc S_m[c][a][b]          (= sum_bc t_ji^bc (mc|ab))
        Buf tpb;
        double* tp = tpb.get(c, OO * VV);   // tp[j][k][d][a] = t_jk^ad
        permute<double>(E, 1.0, "jkad", t, 0.0, "jkda", tp);
        if (!ea) {
            c->Om.alloc(OO * OV, &c->arena);
            c->Pi.alloc(OO * OV, &c->arena);
        }
        long long per_i = (long long)V * V * V;
        long long nI = std::max<long long>(1, (1LL << 30) / (long long)(8 * per_i));
        nI = std::min<long long>(nI, O);
        Buf sb, spb, yb;
        double* S = sb.get(c, (size_t)(nI * per_i));
        double* Sp = spb.get(c, (size_t)(nI * per_i));
        double* Y = yb.get(c, (size_t)(nI * OO * V));
        for (long long i0 = 0; i0 < O; i0 += nI) {
            long long ni = std::min(nI, (long long)O - i0);
            E.ext.extra['I'] = ni;
            ctr<double>(E, 1.0, "IbQ", Bov + i0 * V * Q, "cdQ", Bvv, 0.0, "Ibcd", S);
            permute<double>(E, 1.0, "Icbd", S, 0.0, "Ibcd", Sp);
            axpy<double>(E, -2.0, S, Sp, (size_t)(ni * per_i));
            ctr<double>(E, 1.0, "jkbc", t, "Ibcd", Sp, 0.0, "Ijkd", Y);
            ctr<double>(E, 1.0, "Ijkd", Y, "jkda", tp, 1.0, "Ia", R + i0 * V);
            if (!ea) {
                // Sp2[I][c][d][b] = S[I][c][d][b] - 2 S[I][d][c][b]
                permute<double>(E, -2.0, "Idcb", S, 0.0, "Icdb", Sp);
                axpy<double>(E, 1.0, S, Sp, (size_t)(ni * per_i));
                ctr<double>(E, 1.0, "kjcd", t, "Icdb", Sp, 0.0, "Ikjb", c->Om.p + i0 * OO * V);
                ctr<double>(E, 1.0, "jibc", t, "Icab", S, 0.0, "Ijia", c->Pi.p + i0 * OO * V);
            }
        }
        E.ext.extra.erase('I');
    }
    divide_denom1(E, R, c->eo.p, c->ev.p, O, V, 1.0);   // w = R / (e_i - e_a)

    // ---- transition-moment helpers ------------------------------------------------------
    // omega_kc = s_kc + w_kc + 1/2 s_ld t~_lk^dc
    c->om.alloc(OV, &c->arena);
    ctr<double>(E, 0.5, "ld", c->s.p, "lkdc", tt, 0.0, "kc", c->om.p);
    axpy<double>(E, 1.0, c->s.p, c->om.p, OV);
    axpy<double>(E, 1.0, c->w.p, c->om.p, OV);
    if (ea) {
        // rho_ce += -1/2 t_kl^cd u~_lk^de - 1/2 t_kl^de u~_lk^cd
        ctr<double>(E, -0.5, "klcd", t, "lkde", ut, 1.0, "ce", c->rho.p);
        ctr<double>(E, -0.5, "klde", t, "lkcd", ut, 1.0, "ce", c->rho.p);
    } else {
        // rho_jm += -1/2 t_km^bc u~_jk^cb - 1/2 t_jk^bc u~_km^cb
        ctr<double>(E, -0.5, "kmbc", t, "jkcb", ut, 1.0, "jm", c->rho.p);
        ctr<double>(E, -0.5, "jkbc", t, "kmcb", ut, 1.0, "jm", c->rho.p);
    }
    // t~ + u~ for the 2p1h / 2h1p part of X, and t~ for sigma
    c->ttu.alloc(OO * VV, &c->arena);
    ADC_HIP(hipMemcpyAsync(c->ttu.p, tt, OO * VV * sizeof(double), hipMemcpyDeviceToDevice,
                           E.stream));
    axpy<double>(E, 1.0, ut, c->ttu.p, OO * VV);
    c->tt.alloc(OO * VV, &c->arena);
    ADC_HIP(hipMemcpyAsync(c->tt.p, tt, OO * VV * sizeof(double), hipMemcpyDeviceToDevice,
                           E.stream));
    ADC_HIP(hipStreamSynchronize(E.stream));
}

}  // namespace adc
