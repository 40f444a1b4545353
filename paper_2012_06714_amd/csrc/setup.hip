// Steps 1-3 of Sec. III.A on the device: staging of the DF factors, the
// integral blocks built from them (Eq. 38), MP amplitudes (Eqs. 13-14) and
// the 1p-1p / 1h-1h block, plus the exact diagonal of M in the Z basis.
//
// Resident layouts (row-major, FP64):
//   eo[O], ev[V]
//   Boo[i][j][Q], Bov[i][a][Q], Bvo[a][i][Q], Bvv[a][b][Q]   (B^Q_pq, Q fastest)
//   ovov[i][a][j][b] = (ia|jb)       ooov[i][j][k][a] = (ij|ka)
//   oovv[i][j][a][b] = (ij|ab)       oooo[i][j][k][l] = (ij|kl)   (order 3)
//   t[i][j][a][b]  first-order doubles  t_ij^ab = (ia|jb) / (e_i + e_j - e_a - e_b)
//   s[i][a]        second-order singles
//   u[i][j][a][b]  second-order doubles (order 3)
//   w[i][a]        third-order singles (order 3)
//   M11            EA: [a][b]  IP: [i][j]
#include "context.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace adc {

namespace {

bool is_device_pointer(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

struct Tmp {
    DBuf<double> b;
    double* operator()(adc_ctx* c, size_t n) {
        b.alloc(n, &c->arena);
        return b.p;
    }
};

// t~_ij^ab = 2 t_ij^ab - t_ij^ba
void tilde(adc_ctx* c, const double* t, double* out) {
    Engine& E = c->E;
    permute<double>(E, -1.0, "ijab", t, 0.0, "ijba", out);
    axpy<double>(E, 2.0, t, out, (size_t)c->O * c->O * c->V * c->V);
}

}  // namespace

void setup_all(adc_ctx* c, const double* eps, const double* B) {
    Engine& E = c->E;
    const int O = c->O, V = c->V, Q = c->Q, N = c->N;
    const size_t OO = (size_t)O * O, VV = (size_t)V * V, OV = (size_t)O * V;
    E.ext.O = O;
    E.ext.V = V;
    E.ext.Q = Q;

    // eps and B may be device or host memory (copies of either kind go through
    // hipMemcpyDefault); host B is staged in blocks of auxiliary functions
    c->eo.alloc(O, &c->arena);
    c->ev.alloc(V, &c->arena);
    ADC_HIP(hipMemcpyAsync(c->eo.p, eps, O * sizeof(double), hipMemcpyDefault, E.stream));
    ADC_HIP(hipMemcpyAsync(c->ev.p, eps + O, V * sizeof(double), hipMemcpyDefault, E.stream));
    {
        // energy scale of the learned preconditioner's features: max |eps|
        std::vector<double> h(N);
        ADC_HIP(hipMemcpyAsync(h.data(), eps, N * sizeof(double), hipMemcpyDefault, E.stream));
        ADC_HIP(hipStreamSynchronize(E.stream));
        double s = 0.0;
        for (double v : h) s = std::max(s, std::fabs(v));
        c->escale = s > 0.0 ? s : 1.0;
    }

    // ---- step 1: B blocks (Q fastest) -------------------------------------
    c->Boo.alloc(OO * Q, &c->arena);
    c->Bov.alloc(OV * Q, &c->arena);
    c->Bvv.alloc(VV * Q, &c->arena);
    if (is_device_pointer(B)) {
        stage_block(E, B, Q, N, 0, O, 0, O, c->Boo.p);
        stage_block(E, B, Q, N, 0, O, O, V, c->Bov.p);
        stage_block(E, B, Q, N, O, V, O, V, c->Bvv.p);
    } else {
        // blocks of auxiliary functions through a device buffer of <= 1 GiB
        const long long NN = (long long)N * N;
        const int nq = (int)std::max<long long>(1, std::min<long long>(Q, (1LL << 27) / NN));
        DBuf<double> buf;
        buf.alloc((size_t)(nq * NN), &c->arena);
        for (int q0 = 0; q0 < Q; q0 += nq) {
            const int n = std::min(nq, Q - q0);
            ADC_HIP(hipMemcpyAsync(buf.p, B + (size_t)q0 * NN, (size_t)n * NN * sizeof(double),
                                   hipMemcpyDefault, E.stream));
            stage_block(E, buf.p, n, N, 0, O, 0, O, c->Boo.p, Q, q0);
            stage_block(E, buf.p, n, N, 0, O, O, V, c->Bov.p, Q, q0);
            stage_block(E, buf.p, n, N, O, V, O, V, c->Bvv.p, Q, q0);
            ADC_HIP(hipStreamSynchronize(E.stream));   // the buffer is refilled next
        }
    }
    c->rho.alloc(0, &c->arena);

    c->phase("DF factors staged");
    // integral blocks
    c->ovov.alloc(OV * OV, &c->arena);
    ctr<double>(E, 1.0, "iaQ", c->Bov.p, "jbQ", c->Bov.p, 0.0, "iajb", c->ovov.p);
    c->ooov.alloc(OO * OV, &c->arena);
    ctr<double>(E, 1.0, "ijQ", c->Boo.p, "kaQ", c->Bov.p, 0.0, "ijka", c->ooov.p);

    // ---- step 2: amplitudes ---------------------------------------------------
    c->t.alloc(OO * VV, &c->arena);
    permute<double>(E, 1.0, "iajb", c->ovov.p, 0.0, "ijab", c->t.p);
    divide_denom2(E, c->t.p, c->eo.p, c->ev.p, O, V, 1.0);

    // t~ stays resident (the sigma contractions read it)
    c->tt.alloc(OO * VV, &c->arena);
    double* tt = c->tt.p;
    tilde(c, c->t.p, tt);

    c->phase("first-order doubles");
    // second-order singles: R_ia = -2 t_kl^ca (li|kc) + t_kl^ca (lc|ki) + t~_ik^cd (kd|ac),
    // s = -R / (e_a - e_i)
    c->s.alloc(OV, &c->arena);
    Tmp xb;
    double* X = xb(c, OV * Q);   // X1[i][c][Q] = t~_ik^cd B^Q_kd (reused at third order)
    {
        double* R = c->s.p;
        ctr_sliced<double>(E, -2.0, "klca", c->t.p, "likc", c->ooov.p, 0.0, "ia", R);
        ctr_sliced<double>(E, 1.0, "klca", c->t.p, "kilc", c->ooov.p, 1.0, "ia", R);
        ctr_sliced<double>(E, 1.0, "ikcd", tt, "kdQ", c->Bov.p, 0.0, "icQ", X);
        ctr<double>(E, 1.0, "icQ", X, "acQ", c->Bvv.p, 1.0, "ia", R);
        divide_denom1(E, R, c->eo.p, c->ev.p, O, V, 1.0);
    }

    // ---- step 3: 1p-1p / 1h-1h block through second order ----------------------
    const bool ea = c->kind == ADC_EA;
    const int n1 = c->n1;
    c->M11.alloc((size_t)n1 * n1, &c->arena);
    if (c->m11_fly) {
        // on the fly: M11 keeps only its diagonal through second order,
        // e_a - tau_aa (EA) or -e_i - kappa_ii (IP), for the Davidson correction
        Tmp tb;
        double* td = tb(c, (size_t)n1);
        if (ea) {
            ctr_sliced<double>(E, 2.0, "jkca", c->t.p, "jcka", c->ovov.p, 0.0, "a", td);
            ctr_sliced<double>(E, -1.0, "jkca", c->t.p, "jakc", c->ovov.p, 1.0, "a", td);
        } else {
            ctr_sliced<double>(E, 2.0, "ikbc", c->t.p, "ibkc", c->ovov.p, 0.0, "i", td);
            ctr_sliced<double>(E, -1.0, "ikbc", c->t.p, "ickb", c->ovov.p, 1.0, "i", td);
        }
        std::vector<double> h(n1), e(n1), m((size_t)n1 * n1, 0.0);
        ADC_HIP(hipMemcpyAsync(h.data(), td, n1 * sizeof(double), hipMemcpyDeviceToHost, E.stream));
        ADC_HIP(hipMemcpyAsync(e.data(), ea ? c->ev.p : c->eo.p, n1 * sizeof(double),
                               hipMemcpyDeviceToHost, E.stream));
        ADC_HIP(hipStreamSynchronize(E.stream));
        for (int a = 0; a < n1; ++a) m[(size_t)a * n1 + a] = (ea ? e[a] : -e[a]) - h[a];
        ADC_HIP(hipMemcpyAsync(c->M11.p, m.data(), m.size() * sizeof(double),
                               hipMemcpyHostToDevice, E.stream));
        ADC_HIP(hipStreamSynchronize(E.stream));
    } else {
        Tmp tb;
        double* tau = tb(c, (size_t)n1 * n1);
        if (ea) {
            // tau_ab = t_jk^ca [2 (jc|kb) - (jb|kc)]
            ctr_sliced<double>(E, 2.0, "jkca", c->t.p, "jckb", c->ovov.p, 0.0, "ab", tau);
            ctr_sliced<double>(E, -1.0, "jkca", c->t.p, "jbkc", c->ovov.p, 1.0, "ab", tau);
            symmetrize_m11(E, c->M11.p, tau, c->ev.p, V, 1.0);
        } else {
            // kappa_ij = t_ik^bc [2 (jb|kc) - (jc|kb)]
            ctr_sliced<double>(E, 2.0, "ikbc", c->t.p, "jbkc", c->ovov.p, 0.0, "ij", tau);
            ctr_sliced<double>(E, -1.0, "ikbc", c->t.p, "jckb", c->ovov.p, 1.0, "ij", tau);
            symmetrize_m11(E, c->M11.p, tau, c->eo.p, O, -1.0);
        }
    }

    // spectroscopic-amplitude helper rho (second-order 1p/1h part of T)
    c->rho.alloc((size_t)n1 * n1, &c->arena);
    if (ea) {
        // rho_ce = -1/2 t_kl^de t~_lk^cd
        ctr_sliced<double>(E, -1.0, "klde", c->t.p, "lkcd", c->t.p, 0.0, "ce", c->rho.p);
        ctr_sliced<double>(E, 0.5, "klde", c->t.p, "lkdc", c->t.p, 1.0, "ce", c->rho.p);
    } else {
        // rho_jm = -1/2 t_jk^bc t~_km^cb
        ctr_sliced<double>(E, -1.0, "jkbc", c->t.p, "kmcb", c->t.p, 0.0, "jm", c->rho.p);
        ctr_sliced<double>(E, 0.5, "jkbc", c->t.p, "kmbc", c->t.p, 1.0, "jm", c->rho.p);
    }

    c->phase("second-order singles, 1p-1p / 1h-1h block and rho");
    if (c->order == 3) setup_adc3(c, tt, X);
    else c->tt.release();   // ADC(2) sigma does not read t~

    // IP sigma reads B^Q_ai with the virtual index leading, and never the vv block
    if (!ea) {
        c->Bvo.alloc(OV * Q, &c->arena);
        permute<double>(E, 1.0, "iaQ", c->Bov.p, 0.0, "aiQ", c->Bvo.p);
        c->Bvv.release();
    }

    // ADC(2) needs the (ov|ov) and (oo|ov) blocks only for the amplitudes and
    // M11 above: free them (a batch of systems keeps many contexts resident)
    if (c->order == 2 && !c->m11_fly) {   // (the block applied on the fly reads (ov|ov))
        c->ovov.release();
        c->ooov.release();
    }

    // ---- exact diagonal -------------------------------------------------------
    c->diag.alloc((size_t)c->dim, &c->arena);
    set_diag(E, c->diag.p, c->M11.p, n1);
    if (c->order == 3)
        diag22_first_order(c, c->diag.p);
    else if (ea)
        diag22_adc2(E, c->diag.p, n1, O, V, c->eo.p, c->ev.p, -1.0, 1.0);
    else
        diag22_adc2(E, c->diag.p, n1, V, O, c->ev.p, c->eo.p, 1.0, -1.0);
    ADC_HIP(hipStreamSynchronize(E.stream));
    E.scratch.clear();
    c->phase("diagonal: setup done");
}

}  // namespace adc
