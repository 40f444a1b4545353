// Spectroscopic amplitudes X = T Y and factors P = 2 sum_p X_p^2
// (Eqs. 16, 46-50; step 5 of Sec. III.A).  T is applied from the amplitudes,
// never stored.  For normalised Z-basis vectors, Y = S^{-1/2} Z already
// carries the renormalisation of Eqs. 46-48.
#include "context.hpp"

#include <algorithm>

namespace adc {

static const double SQ3 = 1.7320508075688772;
static const double ALI = 0.5 * (1.0 + 1.0 / SQ3), BEI = 0.5 * (1.0 - 1.0 / SQ3);

void spec_amplitudes(adc_ctx* c, const double* vecs, int nvec, double* Xout) {
    if (c->uhf) {
        spec_amplitudes_uhf(c, vecs, nvec, Xout);
        return;
    }
    Engine& E = c->E;
    E.ext.Z = nvec;
    const int O = c->O, V = c->V, N = c->N, n1 = c->n1, np = (int)c->n2p;
    const long long nx = c->n2x, len2 = nx * np * np, dim = c->dim;
    DBuf<double> y1, y2, xo, xv;
    y1.alloc((size_t)nvec * n1, &c->arena);
    y2.alloc((size_t)nvec * len2, &c->arena);
    xo.alloc((size_t)nvec * O, &c->arena);
    xv.alloc((size_t)nvec * V, &c->arena);
    copy_rows<double, double>(E, vecs, dim, 0, y1.p, n1, 0, nvec, n1, 0.0);
    pair_transform<double, double>(E, vecs, dim, n1, y2.p, len2, 0, nvec, nx, np, ALI, BEI, 0.0);
    const double* t = c->t.p;
    // t~ + u~ contracted over its leading index in blocks copied from host
    // memory when it was parked there (both terms below sum over that index)
    auto ttu_term = [&](const char* sy, const char* st, const char* so, double* out) {
        if (c->ttu.p) {
            ctr<double>(E, 1.0, sy, y2.p, st, c->ttu.p, 0.0, so, out);
            return;
        }
        ADC_REQUIRE(c->ttu_host, "spectroscopic amplitudes: t~ + u~ missing");
        const long long row = (long long)O * V * V;
        const long long nb = std::max<long long>(1, std::min<long long>(O, (1LL << 27) / row));
        DBuf<double> blk;
        blk.alloc((size_t)(nb * row), &c->arena);
        for (long long x0 = 0; x0 < O; x0 += nb) {
            const long long n = std::min(nb, (long long)O - x0);
            ADC_HIP(hipMemcpyAsync(blk.p, c->ttu_host + x0 * row, (size_t)(n * row) * sizeof(double),
                                   hipMemcpyHostToDevice, E.stream));
            ctr_sliced<double>(E, 1.0, sy, y2.p, st, blk.p - x0 * row, x0 == 0 ? 0.0 : 1.0, so, out,
                               {{st[0], x0, n}});
            ADC_HIP(hipStreamSynchronize(E.stream));   // the block buffer is refilled next
        }
    };
    if (c->kind == ADC_EA) {
        // occupied p = k: sum_bcj Y_bcj t~_jk^cb - sum_c Y_c s_kc        (order 2)
        //                 sum_bcj Y_bcj (t~ + u~)_jk^cb - sum_c Y_c omega_kc (order 3)
        if (c->order == 3) {
            ttu_term("zjbc", "jkcb", "zk", xo.p);
            ctr<double>(E, -1.0, "zc", y1.p, "kc", c->om.p, 1.0, "zk", xo.p);
        } else {
            ctr<double>(E, 2.0, "zjbc", y2.p, "jkcb", t, 0.0, "zk", xo.p);
            ctr<double>(E, -1.0, "zjbc", y2.p, "jkbc", t, 1.0, "zk", xo.p);
            ctr<double>(E, -1.0, "zc", y1.p, "kc", c->s.p, 1.0, "zk", xo.p);
        }
        // virtual p = c: Y_c + sum_e rho_ce Y_e
        copy_rows<double, double>(E, y1.p, V, 0, xv.p, V, 0, nvec, V, 0.0);
        ctr<double>(E, 1.0, "ce", c->rho.p, "ze", y1.p, 1.0, "zc", xv.p);
    } else {
        // occupied m: Y_m + sum_j rho_jm Y_j
        copy_rows<double, double>(E, y1.p, O, 0, xo.p, O, 0, nvec, O, 0.0);
        ctr<double>(E, 1.0, "jm", c->rho.p, "zj", y1.p, 1.0, "zm", xo.p);
        // virtual e: sum_jkb Y_jkb t~_kj^be + sum_j Y_j s_je              (order 2)
        //            sum_jkb Y_jkb (t~ + u~)_kj^be + sum_j Y_j omega_je     (order 3)
        if (c->order == 3) {
            ttu_term("zbjk", "kjbe", "ze", xv.p);
            ctr<double>(E, 1.0, "zj", y1.p, "je", c->om.p, 1.0, "ze", xv.p);
        } else {
            ctr<double>(E, 2.0, "zbjk", y2.p, "kjbe", t, 0.0, "ze", xv.p);
            ctr<double>(E, -1.0, "zbjk", y2.p, "kjeb", t, 1.0, "ze", xv.p);
            ctr<double>(E, 1.0, "zj", y1.p, "je", c->s.p, 1.0, "ze", xv.p);
        }
    }
    copy_rows<double, double>(E, xo.p, O, 0, Xout, N, 0, nvec, O, 0.0);
    copy_rows<double, double>(E, xv.p, V, 0, Xout, N, O, nvec, V, 0.0);
    ADC_HIP(hipStreamSynchronize(E.stream));
}

}  // namespace adc
