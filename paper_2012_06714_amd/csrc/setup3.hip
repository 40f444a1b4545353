// Third-order additions to the setup: second-order doubles u through the
// particle-particle ladder Lambda (rebuilt from B like the sigma vvvv term),
// third-order singles w, the third-order 1p-1p (EA) or 1h-1h (IP) block and the
// intermediates of the second-order coupling (Gamma; for IP also the
// precontracted Omega and Pi blocks) and of the transition moments.
//
// Notation: t~ = 2 t_ij^ab - t_ij^ba (same for u~, Lambda~); (pq|rs) from the
// resident blocks or as sum_Q B B; every contraction is named by its einsum
// string.  All of it runs once, in FP64.
//
// Memory: besides the resident (ov|ov), (oo|vv), t and t~, at most the second-
// order doubles u and one more O^2 V^2 tensor (u~, later t~ + u~) exist at a
// time.  Every other four-index intermediate (the ring, hole-hole and
// t t~ products, D u, the B-sized (Pt B) and (B s) products) is made one block
// of its leading index at a time and contracted at once; contractions over
// large operands go through ctr_sliced, whose temporaries stay within the
// engine's slice budget.  The sums are those of the full tensors, in blocks.
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

// A block buffer holding rows [x0, x0 + n) of a tensor whose leading axis has
// extent `full` and `row` elements per leading index, addressed as the full
// tensor (the returned pointer minus x0 rows): ctr_sliced reads and writes it
// only inside the slice of that leading letter.
double* block_view(double* buf, long long x0, long long row) { return buf - x0 * row; }

// block length along an occupied index so that a block of rows of `row`
// elements stays within the slice budget
long long occ_block(const adc_ctx* c, long long row) {
    const long long nb = std::max<long long>(1, c->E.slice_budget / std::max<long long>(1, row));
    return std::min<long long>(nb, c->O);
}
}  // namespace

using Sl = std::vector<Slice>;

// third-order terms of the 1p-1p block (EA) that read u, the rings and the
// hole-hole ladder; M holds the lower orders on entry
static void m11_third_ea(adc_ctx* c, double* M, const double* t, const double* tt,
                         const double* u, const double* P) {
    Engine& E = c->E;
    const int O = c->O, V = c->V, Q = c->Q;
    const long long OV = (long long)O * V, VV = (long long)V * V, OVV = OV * V;
    const double *Bov = c->Bov.p, *Bvv = c->Bvv.p, *ovov = c->ovov.p, *oovv = c->oovv.p,
                 *oooo = c->oooo.p;
    Buf Tb, Wb;
    double* T = Tb.get(c, VV);
    double* v = Wb.get(c, (size_t)Q);
    // -1/2 (tau[u] + tau[u]^T), tau_ab = u_jk^ca [2 (jc|kb) - (jb|kc)]
    ctr_sliced<double>(E, 2.0, "jkca", u, "jckb", ovov, 0.0, "ab", T);
    ctr_sliced<double>(E, -1.0, "jkca", u, "jbkc", ovov, 1.0, "ab", T);
    permute<double>(E, -0.5, "ab", T, 1.0, "ab", M);
    permute<double>(E, -0.5, "ba", T, 1.0, "ab", M);
    // s terms: 4 (jc|ab) s_jc - (jb|ac) s_jc - (ja|bc) s_jc; the second through
    // Ys[b][c][Q] = sum_j B^Q_jb s_jc, one block of b at a time
    ctr<double>(E, 1.0, "jc", c->s.p, "jcQ", Bov, 0.0, "Q", v);
    ctr<double>(E, 4.0, "abQ", Bvv, "Q", v, 1.0, "ab", M);
    {
        const long long row = (long long)V * Q;
        const long long nb = std::max<long long>(1, std::min<long long>(V, E.slice_budget / row));
        Buf Ysb;
        double* Ys = Ysb.get(c, (size_t)(nb * row));
        for (long long b0 = 0; b0 < V; b0 += nb) {
            const Sl sb{{'b', b0, std::min(nb, V - b0)}};
            double* Ysv = block_view(Ys, b0, row);
            ctr_sliced<double>(E, 1.0, "jbQ", Bov, "jc", c->s.p, 0.0, "bcQ", Ysv, sb);
            ctr_sliced<double>(E, 1.0, "acQ", Bvv, "bcQ", Ysv, 0.0, "ab", T, sb);
        }
    }
    permute<double>(E, -1.0, "ab", T, 1.0, "ab", M);
    permute<double>(E, -1.0, "ba", T, 1.0, "ab", M);
    // -1/2 (pi + pi^T), pi_ae = t~_jk^ba Du_jk^be with Du = (e_b + e_e - e_j - e_k) u,
    // D u made one block of j at a time
    {
        const long long nj = occ_block(c, OVV);
        Buf Db;
        double* Du = Db.get(c, (size_t)(nj * OVV));
        for (long long j0 = 0; j0 < O; j0 += nj) {
            const long long n = std::min(nj, (long long)O - j0);
            mul_denom2(E, u + j0 * OVV, Du, c->eo.p, c->ev.p, O, V, (int)j0, (int)n);
            ctr_sliced<double>(E, 1.0, "jkba", tt, "jkbe", block_view(Du, j0, OVV),
                               j0 == 0 ? 0.0 : 1.0, "ae", T, Sl{{'j', j0, n}});
        }
    }
    permute<double>(E, -0.5, "ab", T, 1.0, "ab", M);
    permute<double>(E, -0.5, "ba", T, 1.0, "ab", M);

    const long long nb = occ_block(c, OVV);
    Buf b1, b2, b3, b4;
    double* X1 = b1.get(c, (size_t)(nb * OVV));
    double* X2 = b2.get(c, (size_t)(nb * OVV));
    double* X3 = b3.get(c, (size_t)(nb * OVV));
    double* X4 = b4.get(c, (size_t)(nb * OVV));
    for (long long k0 = 0; k0 < O; k0 += nb) {
        c->phase("third-order 1p-1p: rings, block", k0, O);
        const long long n = std::min(nb, (long long)O - k0);
        double* Z = block_view(X1, k0, OVV);
        // hole-hole ladder Zo_kj^ca = (mk|lj) t_lm^ca, block of its first index:
        //   + t_jk^cb Zo_jk^ca - 2 t_jk^cb Zo_kj^ca
        ctr_sliced<double>(E, 1.0, "mklj", oooo, "lmca", t, 0.0, "kjca", Z, Sl{{'k', k0, n}});
        ctr_sliced<double>(E, 1.0, "jkcb", t, "jkca", Z, 1.0, "ab", M, Sl{{'j', k0, n}});
        ctr_sliced<double>(E, -2.0, "jkcb", t, "kjca", Z, 1.0, "ab", M, Sl{{'k', k0, n}});
        // rings R[j][c][k][a] = t~_lj^dc (ld|ka) (R1), t~_lj^dc (lk|ad) (R2),
        // t~_lj^cd (lk|ad) (R3), block of j
        const Sl sj{{'j', k0, n}};
        double* R1 = block_view(X2, k0, OVV);
        double* R2 = block_view(X3, k0, OVV);
        double* R3 = block_view(X4, k0, OVV);
        ctr_sliced<double>(E, 1.0, "ljdc", tt, "ldka", ovov, 0.0, "jcka", R1, sj);
        ctr_sliced<double>(E, 1.0, "ljdc", tt, "lkad", oovv, 0.0, "jcka", R2, sj);
        ctr_sliced<double>(E, 1.0, "ljcd", tt, "lkad", oovv, 0.0, "jcka", R3, sj);
        ctr_sliced<double>(E, -1.0, "jkcb", tt, "jcka", R1, 1.0, "ab", M, sj);
        ctr_sliced<double>(E, 1.0, "jkcb", t, "jcka", R2, 1.0, "ab", M, sj);
        ctr_sliced<double>(E, 1.0, "jkbc", t, "jcka", R3, 1.0, "ab", M, sj);
        // R3 + R1 and R2 - 2 R1 (in the buffers of R3 and R2)
        axpy<double>(E, 1.0, X2, X4, (size_t)(n * OVV));
        axpy<double>(E, -2.0, X2, X3, (size_t)(n * OVV));
        ctr_sliced<double>(E, 1.0, "jkcb", t, "jakc", R3, 1.0, "ab", M, sj);
        ctr_sliced<double>(E, 1.0, "jkbc", t, "jakc", R2, 1.0, "ab", M, sj);
        // Q5 = t~_jk^cd t_lj^da + t~_jk^dc t_lj^ad ; Q6 = t~_jk^dc t~_lj^ad  ([k][c][l][a]),
        // block of k:  + Q5 (lk|cb) - Q6 (lb|kc)
        const Sl sk{{'k', k0, n}};
        double* Q5 = block_view(X1, k0, OVV);
        double* Q6 = block_view(X2, k0, OVV);
        ctr_sliced<double>(E, 1.0, "jkcd", tt, "ljda", t, 0.0, "kcla", Q5, sk);
        ctr_sliced<double>(E, 1.0, "jkdc", tt, "ljad", t, 1.0, "kcla", Q5, sk);
        ctr_sliced<double>(E, 1.0, "jkdc", tt, "ljad", tt, 0.0, "kcla", Q6, sk);
        ctr_sliced<double>(E, 1.0, "kcla", Q5, "lkcb", oovv, 1.0, "ab", M, sk);
        ctr_sliced<double>(E, -1.0, "kcla", Q6, "lbkc", ovov, 1.0, "ab", M, sk);
    }
    ctr_sliced<double>(E, 1.0, "kl", P, "lbka", ovov, 1.0, "ab", M);
    ctr_sliced<double>(E, -2.0, "kl", P, "lkab", oovv, 1.0, "ab", M);
}

// third-order terms of the 1h-1h block (IP) that read u, the rings and the
// t t~ products; M holds the lower orders on entry
static void m11_third_ip(adc_ctx* c, double* M, const double* t, const double* tt,
                         const double* u, const double* P, const double* P7, const double* Pt) {
    Engine& E = c->E;
    const int O = c->O, V = c->V;
    const long long OV = (long long)O * V, OVV = OV * V, OO = (long long)O * O;
    const double *ooov = c->ooov.p, *ovov = c->ovov.p, *oovv = c->oovv.p, *oooo = c->oooo.p;
    Buf Tb, Mtb;
    double* T = Tb.get(c, OO);
    double* Mt = Mtb.get(c, OO);   // terms computed transposed, added as Mt^T at the end
    fill<double>(E, Mt, 0.0, OO);
    // -1/2 (kappa[u] + kappa[u]^T), kappa_ij = u_ik^bc [2 (jb|kc) - (jc|kb)]
    ctr_sliced<double>(E, 2.0, "ikbc", u, "jbkc", ovov, 0.0, "ij", T);
    ctr_sliced<double>(E, -1.0, "ikbc", u, "jckb", ovov, 1.0, "ij", T);
    permute<double>(E, -0.5, "ij", T, 1.0, "ij", M);
    permute<double>(E, -0.5, "ji", T, 1.0, "ij", M);
    // s terms
    ctr<double>(E, -4.0, "kb", c->s.p, "jikb", ooov, 1.0, "ij", M);
    ctr<double>(E, 1.0, "kb", c->s.p, "kijb", ooov, 1.0, "ij", M);
    ctr<double>(E, 1.0, "kb", c->s.p, "jkib", ooov, 1.0, "ij", M);
    // -1/2 (pi + pi^T), pi_ij = t~_ik^bc Du_jk^bc, D u one block of j at a time
    {
        const long long nj = occ_block(c, OVV);
        Buf Db;
        double* Du = Db.get(c, (size_t)(nj * OVV));
        fill<double>(E, T, 0.0, OO);
        for (long long j0 = 0; j0 < O; j0 += nj) {
            const long long n = std::min(nj, (long long)O - j0);
            mul_denom2(E, u + j0 * OVV, Du, c->eo.p, c->ev.p, O, V, (int)j0, (int)n);
            ctr_sliced<double>(E, 1.0, "ikbc", tt, "jkbc", block_view(Du, j0, OVV), 1.0, "ij", T,
                               Sl{{'j', j0, n}});
        }
    }
    permute<double>(E, -0.5, "ij", T, 1.0, "ij", M);
    permute<double>(E, -0.5, "ji", T, 1.0, "ij", M);
    // hole-hole pieces
    ctr<double>(E, -2.0, "jklm", P7, "milk", oooo, 1.0, "ij", M);
    ctr<double>(E, 1.0, "jklm", P7, "mkli", oooo, 1.0, "ij", M);
    ctr<double>(E, -2.0, "iklm", P7, "jmkl", oooo, 1.0, "ij", M);
    ctr<double>(E, 1.0, "iklm", P7, "jlkm", oooo, 1.0, "ij", M);
    ctr<double>(E, 2.0, "lm", P, "jiml", oooo, 1.0, "ij", M);
    ctr<double>(E, -1.0, "lm", P, "jlmi", oooo, 1.0, "ij", M);
    const long long nb = occ_block(c, OVV);
    Buf b1, b2, b3;
    double* X1 = b1.get(c, (size_t)(nb * OVV));
    double* X2 = b2.get(c, (size_t)(nb * OVV));
    double* X3 = b3.get(c, (size_t)(nb * OVV));
    for (long long j0 = 0; j0 < O; j0 += nb) {
        c->phase("third-order 1h-1h: rings, block", j0, O);
        const long long n = std::min(nb, (long long)O - j0);
        // rings with Ra = R2 - 2 R1 and Rb = R3 + R1 ([j][c][k][a], block of j)
        const Sl sj{{'j', j0, n}};
        double* R1 = block_view(X1, j0, OVV);
        double* Ra = block_view(X2, j0, OVV);
        double* Rb = block_view(X3, j0, OVV);
        ctr_sliced<double>(E, 1.0, "ljdc", tt, "ldka", ovov, 0.0, "jcka", R1, sj);
        ctr_sliced<double>(E, 1.0, "ljdc", tt, "lkad", oovv, 0.0, "jcka", Ra, sj);
        ctr_sliced<double>(E, 1.0, "ljcd", tt, "lkad", oovv, 0.0, "jcka", Rb, sj);
        axpy<double>(E, -2.0, X1, X2, (size_t)(n * OVV));
        axpy<double>(E, 1.0, X1, X3, (size_t)(n * OVV));
        // the ring index named k below is the block's first index
        const Sl sk{{'k', j0, n}};
        ctr_sliced<double>(E, 1.0, "jkbc", t, "kcib", Ra, 1.0, "ij", M, sk);
        ctr_sliced<double>(E, 1.0, "jkbc", t, "kbic", Rb, 1.0, "ij", M, sk);
        // t_ik^bc Ra_jbkc and t_ik^bc Rb_jckb, accumulated transposed ([j][i])
        ctr_sliced<double>(E, 1.0, "ikbc", t, "jbkc", Ra, 1.0, "ji", Mt, sj);
        ctr_sliced<double>(E, 1.0, "ikbc", t, "jckb", Rb, 1.0, "ji", Mt, sj);
        // Q7 = t_ik^bc t~_kl^db, Q8 = t_ik^bc t~_kl^bd ([i][c][l][d]),
        // Q9 = t_ik^bc t~_kl^cd ([i][b][l][d]); block of i
        const Sl si{{'i', j0, n}};
        double* Qx = block_view(X1, j0, OVV);
        ctr_sliced<double>(E, 1.0, "ikbc", t, "kldb", tt, 0.0, "icld", Qx, si);
        ctr_sliced<double>(E, 1.0, "icld", Qx, "jldc", oovv, 1.0, "ij", M, si);
        ctr_sliced<double>(E, 1.0, "ikbc", t, "klbd", tt, 0.0, "icld", Qx, si);
        ctr_sliced<double>(E, 1.0, "icld", Qx, "jcld", ovov, 1.0, "ij", M, si);
        ctr_sliced<double>(E, 1.0, "ikbc", t, "klcd", tt, 0.0, "ibld", Qx, si);
        ctr_sliced<double>(E, 1.0, "ibld", Qx, "jldb", oovv, 1.0, "ij", M, si);
        ctr_sliced<double>(E, -2.0, "ibld", Qx, "jbld", ovov, 1.0, "ij", M, si);
    }
    permute<double>(E, 1.0, "ji", Mt, 1.0, "ij", M);
    ctr_sliced<double>(E, 1.0, "bd", Pt, "jdib", ovov, 1.0, "ij", M);
    ctr_sliced<double>(E, -2.0, "bd", Pt, "jibd", oovv, 1.0, "ij", M);
}

void setup_adc3(adc_ctx* c, const double* tt, const double* X1) {
    const bool ea = c->kind == ADC_EA;
    Engine& E = c->E;
    const int O = c->O, V = c->V, Q = c->Q;
    const size_t OO = (size_t)O * O, VV = (size_t)V * V, OV = (size_t)O * V;
    const long long OVV = (long long)OV * V;
    const double* t = c->t.p;
    const double *Bov = c->Bov.p, *Bvv = c->Bvv.p, *Boo = c->Boo.p;
    const double *ovov = c->ovov.p, *ooov = c->ooov.p;

    c->oovv.alloc(OO * VV, &c->arena);
    ctr<double>(E, 1.0, "ijQ", Boo, "abQ", Bvv, 0.0, "ijab", c->oovv.p);
    c->oooo.alloc(OO * OO, &c->arena);
    ctr<double>(E, 1.0, "ijQ", Boo, "klQ", Boo, 0.0, "ijkl", c->oooo.p);
    const double *oovv = c->oovv.p, *oooo = c->oooo.p;
    double* M = c->M11.p;

    // third-order singles w: its terms are accumulated in R (= w) as their
    // operands become available, divided by the denominators at the end
    c->w.alloc(OV, &c->arena);
    double* R = c->w.p;
    fill<double>(E, R, 0.0, OV);

    // ---- Gamma_jb = G_bj + H_bj + Ds_jb -------------------------------------------
    //   G_bj = t_kl^cb [(jk|cl) - 2 (jl|ck)],  H_bj = t~_jk^cd [2 (dk|cb) - (db|ck)] = X1 . Bvv
    Buf Gb, Dsb;
    double* G = Gb.get(c, OV);
    ctr_sliced<double>(E, 1.0, "klcb", t, "jklc", ooov, 0.0, "jb", G);
    ctr_sliced<double>(E, -2.0, "klcb", t, "jlkc", ooov, 1.0, "jb", G);
    double* Ds = Dsb.get(c, OV);
    mul_denom1(E, c->s.p, Ds, c->eo.p, c->ev.p, O, V);
    c->gam.alloc(OV, &c->arena);
    ctr<double>(E, 1.0, "jcQ", X1, "cbQ", Bvv, 0.0, "jb", c->gam.p);
    axpy<double>(E, 1.0, G, c->gam.p, OV);
    axpy<double>(E, 1.0, Ds, c->gam.p, OV);

    c->phase("(oo|vv), (oo|oo), Gamma");
    // ---- shared intermediates ----------------------------------------------------------
    const bool fly = c->m11_fly;   // the 1p-1p / 1h-1h block is applied on the fly
    c->P.alloc(OO, &c->arena);
    double* P = c->P.p;                      // P_kl = t_jk^cd t~_lj^dc
    ctr_sliced<double>(E, 1.0, "jkcd", t, "ljdc", tt, 0.0, "kl", P);
    c->P7.alloc(OO * OO, &c->arena);
    double* P7 = c->P7.p;                    // P7_ijkl = t_ij^bc t_kl^cb
    ctr_sliced<double>(E, 1.0, "ijbc", t, "klcb", t, 0.0, "ijkl", P7);
    c->Pt.alloc(VV, &c->arena);
    double* Pt = c->Pt.p;                    // Pt_ce = t_jk^cd t~_kj^de
    ctr_sliced<double>(E, 1.0, "jkcd", t, "kjde", tt, 0.0, "ce", Pt);
    c->wq.alloc((size_t)Q, &c->arena);
    double* wq = c->wq.p;                    // sum_ce Pt_ce B^Q_ce
    ctr<double>(E, 1.0, "ce", Pt, "ceQ", Bvv, 0.0, "Q", wq);
    {
        // Zp[a][c][Q] = Pt_ce B^Q_ae, one block of a at a time:
        //   EA M11: - Zp(ac|Q) B^Q_bc;  w: - B^Q_ib Zp[a][b][Q]
        const long long row = (long long)V * Q;
        const long long na = std::max<long long>(1, std::min<long long>(V, E.slice_budget / row));
        Buf Zpb;
        double* Zp = Zpb.get(c, (size_t)(na * row));
        for (long long a0 = 0; a0 < V; a0 += na) {
            const Sl sa{{'a', a0, std::min(na, V - a0)}};
            double* Zv = block_view(Zp, a0, row);
            ctr_sliced<double>(E, 1.0, "aeQ", Bvv, "ce", Pt, 0.0, "acQ", Zv, sa);
            if (ea && !fly) ctr_sliced<double>(E, -1.0, "acQ", Zv, "bcQ", Bvv, 1.0, "ab", M, sa);
            ctr_sliced<double>(E, -1.0, "ibQ", Bov, "abQ", Zv, 1.0, "ia", R, sa);
        }
    }
    if (ea && !fly) ctr<double>(E, 2.0, "abQ", Bvv, "Q", wq, 1.0, "ab", M);   // 2 Pt.(ce|ab)

    c->phase("P, P7, Pt and the Pt B terms");
    // ---- particle-particle ladder and second-order doubles --------------------------
    // Lambda_ij^ab = (ac|bd) t_ij^cd, written into u's buffer; t_ij^cd = t_ji^dc, so the
    // mirrored products are rows of the direct ones
    c->u.alloc(OO * VV, &c->arena);
    double* u = c->u.p;
    vvvv_apply<double, double>(c, Bvv, t, u, (long long)OO, O);
    E.scratch.clear();   // the rebuilt slab and operand copies are not needed again here
    c->phase("particle-particle ladder");
    // third-order 1p-1p / 1h-1h terms through Lambda~ = 2 Lambda - Lambda^(ab):
    //   EA: - t_jk^cb Lambda~_jk^ca - t_jk^ac Lambda~_jk^bc;  IP: - t_ik^bc Lambda~_jk^bc
    // (on the fly: Lambda kept instead)
    if (fly) {
        c->Lam.alloc(OO * VV, &c->arena);
        ADC_HIP(hipMemcpyAsync(c->Lam.p, u, OO * VV * sizeof(double), hipMemcpyDeviceToDevice,
                               E.stream));
    } else if (ea) {
        ctr_sliced<double>(E, -2.0, "jkcb", t, "jkca", u, 1.0, "ab", M);
        ctr_sliced<double>(E, 1.0, "jkcb", t, "jkac", u, 1.0, "ab", M);
        ctr_sliced<double>(E, -2.0, "jkac", t, "jkbc", u, 1.0, "ab", M);
        ctr_sliced<double>(E, 1.0, "jkac", t, "jkcb", u, 1.0, "ab", M);
    } else {
        ctr_sliced<double>(E, -2.0, "ikbc", t, "jkbc", u, 1.0, "ij", M);
        ctr_sliced<double>(E, 1.0, "ikbc", t, "jkcb", u, 1.0, "ij", M);
    }
    // u = [Lambda + hole-hole ladder + rings] / (e_i + e_j - e_a - e_b)
    ctr_sliced<double>(E, 1.0, "klba", t, "likj", oooo, 1.0, "ijab", u);
    ctr_sliced<double>(E, -1.0, "jkca", t, "kibc", oovv, 1.0, "ijab", u);
    ctr_sliced<double>(E, -1.0, "jkbc", t, "kiac", oovv, 1.0, "ijab", u);
    ctr_sliced<double>(E, -1.0, "ikac", t, "kjbc", oovv, 1.0, "ijab", u);
    ctr_sliced<double>(E, -1.0, "ikcb", t, "kjac", oovv, 1.0, "ijab", u);
    ctr_sliced<double>(E, 1.0, "jkbc", tt, "kcia", ovov, 1.0, "ijab", u);
    ctr_sliced<double>(E, 1.0, "ikac", tt, "kcjb", ovov, 1.0, "ijab", u);
    divide_denom2(E, u, c->eo.p, c->ev.p, O, V, 1.0);
    E.scratch.clear();
    c->phase("second-order doubles");

    // ---- third-order 1p-1p / 1h-1h block -------------------------------------------------
    if (fly) {
        c->Du.alloc(OO * VV, &c->arena);    // (e_a + e_b - e_i - e_j) u, read on the fly
        mul_denom2(E, u, c->Du.p, c->eo.p, c->ev.p, O, V);
    } else if (ea) {
        m11_third_ea(c, M, t, tt, u, P);
    } else {
        m11_third_ip(c, M, t, tt, u, P, P7, Pt);
    }
    E.scratch.clear();
    c->phase("third-order 1p-1p / 1h-1h block");

    // ---- third-order singles w (the Zp term is already in R) ----------------------------
    ctr_sliced<double>(E, 1.0, "jkba", u, "jikb", ooov, 1.0, "ia", R);
    ctr_sliced<double>(E, -2.0, "jkba", u, "kijb", ooov, 1.0, "ia", R);
    ctr_sliced<double>(E, -1.0, "jb", c->s.p, "jiab", oovv, 1.0, "ia", R);
    ctr_sliced<double>(E, 3.0, "jb", c->s.p, "jbia", ovov, 1.0, "ia", R);
    ctr_sliced<double>(E, -0.5, "jb", c->s.p, "ibja", ovov, 1.0, "ia", R);
    // u~ (its buffer becomes t~ + u~ below)
    c->ttu.alloc(OO * VV, &c->arena);
    double* ut = c->ttu.p;
    tilde_of(c, u, ut);
    if (!fly) c->u.release();   // u is read only through u~ from here on
    {
        Buf x2b;
        double* X2 = x2b.get(c, OV * Q);
        ctr_sliced<double>(E, 1.0, "ijbc", ut, "jcQ", Bov, 0.0, "ibQ", X2);
        ctr<double>(E, 1.0, "ibQ", X2, "abQ", Bvv, 1.0, "ia", R);
        // t~ (Gamma - Ds/2)
        Buf gb;
        double* gmh = gb.get(c, OV);
        ADC_HIP(hipMemcpyAsync(gmh, c->gam.p, OV * sizeof(double), hipMemcpyDeviceToDevice,
                               E.stream));
        axpy<double>(E, -0.5, Ds, gmh, OV);
        ctr_sliced<double>(E, 1.0, "ijab", tt, "jb", gmh, 1.0, "ia", R);
        // P_kl [(li|ka) - 2 (lk|ia)]
        ctr<double>(E, 1.0, "kl", P, "lika", ooov, 1.0, "ia", R);
        ctr<double>(E, -2.0, "kl", P, "lkia", ooov, 1.0, "ia", R);
        // PA, PB ([k][b][l][a]), PC ([k][c][l][a]), one block of k at a time
        const long long nb = occ_block(c, OVV);
        Buf pb;
        double* PX = pb.get(c, (size_t)(nb * OVV));
        for (long long k0 = 0; k0 < O; k0 += nb) {
            c->phase("third-order singles: t t~ products, block", k0, O);
            const Sl sk{{'k', k0, std::min(nb, (long long)O - k0)}};
            double* Pv = block_view(PX, k0, OVV);
            ctr_sliced<double>(E, 1.0, "jkbc", t, "ljac", tt, 0.0, "kbla", Pv, sk);
            ctr_sliced<double>(E, 1.0, "kbla", Pv, "likb", ooov, 1.0, "ia", R, sk);
            ctr_sliced<double>(E, 1.0, "jkbc", t, "ljca", tt, 0.0, "kbla", Pv, sk);
            ctr_sliced<double>(E, 1.0, "kbla", Pv, "lkib", ooov, 1.0, "ia", R, sk);
            ctr_sliced<double>(E, 1.0, "jkbc", t, "ljab", tt, 0.0, "kcla", Pv, sk);
            ctr_sliced<double>(E, 1.0, "kcla", Pv, "lkic", ooov, 1.0, "ia", R, sk);
            ctr_sliced<double>(E, -2.0, "kcla", Pv, "likc", ooov, 1.0, "ia", R, sk);
        }
        // P7 [2 (jk|la) - (jl|ka)]
        ctr<double>(E, -1.0, "ijkl", P7, "jlka", ooov, 1.0, "ia", R);
        ctr<double>(E, 2.0, "ijkl", P7, "jkla", ooov, 1.0, "ia", R);
        // Pt term: 2 Pt.(bd|ai)
        ctr<double>(E, 2.0, "Q", wq, "iaQ", Bov, 1.0, "ia", R);
        // t~ X1 Bvv
        ctr_sliced<double>(E, 1.0, "ijbc", tt, "jcQ", X1, 0.0, "ibQ", X2);
        ctr<double>(E, 1.0, "ibQ", X2, "abQ", Bvv, 1.0, "ia", R);
        // Pq[i][c][k][d] = t_ij^bc t~_jk^db + t_ij^cb t~_jk^bd ; -(dc|ak), through
        // Tq[i][k][Q] = Pq (cd|Q), one block of i at a time
        Buf tqb;
        double* Tq = tqb.get(c, OO * Q);
        for (long long i0 = 0; i0 < O; i0 += nb) {
            const Sl si{{'i', i0, std::min(nb, (long long)O - i0)}};
            double* Pv = block_view(PX, i0, OVV);
            ctr_sliced<double>(E, 1.0, "ijbc", t, "jkdb", tt, 0.0, "ickd", Pv, si);
            ctr_sliced<double>(E, 1.0, "ijcb", t, "jkbd", tt, 1.0, "ickd", Pv, si);
            ctr_sliced<double>(E, 1.0, "ickd", Pv, "cdQ", Bvv, 0.0, "ikQ", Tq, si);
        }
        ctr<double>(E, -1.0, "ikQ", Tq, "kaQ", Bov, 1.0, "ia", R);
    }
    E.scratch.clear();
    c->phase("third-order singles: amplitude terms");
    {
        // slabs S_m[b][c][d] = (b m|c d), m in a block of occupied orbitals:
        //   w:  R_ma += sum_jkd [sum_bc t_jk^bc (S_m[c][b][d] - 2 S_m[b][c][d])] t_jk^ad
        //       (the inner sum stored as Y[m][k][j][d]; t_jk^ad = t_kj^da is t's own layout)
        //   IP: Omega[m][k][j][b] = t_kj^cd (S_m[c][d][b] - 2 S_m[d][c][b])
        //       Pi[m][j][i][a]    = t_ji^bc S_m[c][a][b]          (= sum_bc t_ji^bc (mc|ab))
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
            c->phase("(vv|vo) slab", i0, O);
            long long ni = std::min(nI, (long long)O - i0);
            E.ext.extra['I'] = ni;
            ctr<double>(E, 1.0, "IbQ", Bov + i0 * V * Q, "cdQ", Bvv, 0.0, "Ibcd", S);
            permute<double>(E, 1.0, "Icbd", S, 0.0, "Ibcd", Sp);
            axpy<double>(E, -2.0, S, Sp, (size_t)(ni * per_i));
            ctr<double>(E, 1.0, "jkbc", t, "Ibcd", Sp, 0.0, "Ikjd", Y);
            ctr<double>(E, 1.0, "Ikjd", Y, "kjda", t, 1.0, "Ia", R + i0 * V);
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
    c->phase("third-order singles: (vv|vo) slabs");

    // ---- transition-moment helpers ------------------------------------------------------
    // omega_kc = s_kc + w_kc + 1/2 s_ld t~_lk^dc
    c->om.alloc(OV, &c->arena);
    ctr_sliced<double>(E, 0.5, "ld", c->s.p, "lkdc", tt, 0.0, "kc", c->om.p);
    axpy<double>(E, 1.0, c->s.p, c->om.p, OV);
    axpy<double>(E, 1.0, c->w.p, c->om.p, OV);
    if (ea) {
        // rho_ce += -1/2 t_kl^cd u~_lk^de - 1/2 t_kl^de u~_lk^cd
        ctr_sliced<double>(E, -0.5, "klcd", t, "lkde", ut, 1.0, "ce", c->rho.p);
        ctr_sliced<double>(E, -0.5, "klde", t, "lkcd", ut, 1.0, "ce", c->rho.p);
    } else {
        // rho_jm += -1/2 t_km^bc u~_jk^cb - 1/2 t_jk^bc u~_km^cb
        ctr_sliced<double>(E, -0.5, "kmbc", t, "jkcb", ut, 1.0, "jm", c->rho.p);
        ctr_sliced<double>(E, -0.5, "jkbc", t, "kmcb", ut, 1.0, "jm", c->rho.p);
    }
    // t~ + u~ for the 2p1h / 2h1p part of X
    axpy<double>(E, 1.0, tt, c->ttu.p, OO * VV);
    if (!fly) {   // the small intermediates are read again only on the fly
        c->P.release();
        c->P7.release();
        c->Pt.release();
        c->wq.release();
    }
    E.scratch.clear();
    ADC_HIP(hipStreamSynchronize(E.stream));
}

}  // namespace adc
