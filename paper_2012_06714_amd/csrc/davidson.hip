// Block Davidson-Liu eigensolver with an FP64 subspace (step 4 of Sec. III.A;
// the paper uses a multiroot Davidson solver).  Basis V and sigma vectors W
// stay on the device; the projected matrix G = V W^T is diagonalised with
// rocSOLVER; only Ritz values and residual norms (a few hundred bytes) cross
// to the host each iteration.
//
// Parameters follow this reading of the method:
//   guesses: unit vectors at the `block` smallest diagonal entries (ties to the
//            lower index) or the vectors given by adc_set_guess;
//   converged when every root k < nroots has |theta_k - theta_k(prev)| <=
//            max(tol_e, 8 eps |theta_k|) (eps the FP64 unit roundoff: no
//            change below the resolution of theta is meaningful) and
//            ||r_k|| <= tol_r max(1, |theta_k|) (the residual bound is
//            relative for roots beyond 1 Eh, absolute otherwise);
//   correction d = r / (theta - D) with |theta - D| floored at 1e-8, or the
//            learned correction of it (mlp.hip) when a network is installed;
//   new directions (scaled to unit norm) are orthogonalised against V by block
//            Gram-Schmidt and among themselves through their Gram matrix, in
//            two passes; directions whose Gram eigenvalue falls below
//            max(1e-20, 1e-14 lambda_max) are dropped;
//   restart to the current `block` Ritz vectors when V would exceed max_space.
// Mixed precision ("precision" = 1): sigma runs with BF16 products until the
// (scaled) residuals fall below max(sqrt(tol_r), 1e-3) or 3e-3, or stop
// decreasing (three iterations without a 10% decrease); the space is then
// rebuilt from the Ritz vectors with FP64 sigma
// and the iteration continues in FP64 to the requested tolerance (iterative
// refinement of the reduced-precision subspace).  "precision" = 2 inserts a
// phase with FP32 products between the two, left at scaled residuals of
// max(tol_r, 2e-6) or when they stop decreasing.
#include "context.hpp"

#include <rocsolver/rocsolver.h>

#include "syev_host.hpp"

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <numeric>

namespace adc {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// part[k][b] = sum over chunk b of row k of x^2  (wavefront shuffles + LDS)
__global__ void k_rownorm_part(const double* __restrict__ R, long long dim, int nchunk,
                               double* __restrict__ part) {
    const int k = blockIdx.y, b = blockIdx.x;
    const long long chunk = (dim + nchunk - 1) / nchunk;
    const long long lo = b * chunk, hi = min(dim, lo + chunk);
    double acc = 0.0;
    for (long long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double v = R[(long long)k * dim + e];
        acc += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double red[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        part[(long long)k * nchunk + b] = s;
    }
}

__global__ void k_rownorm_final(const double* part, int nchunk, int nrow, double* out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nrow) {
        double s = 0.0;
        for (int b = 0; b < nchunk; ++b) s += part[(long long)k * nchunk + b];
        out[k] = sqrt(s);
    }
}

// R[k] = AX[k] - theta[k] X[k]
__global__ void k_residual(const double* __restrict__ AX, const double* __restrict__ X,
                           const double* __restrict__ theta, double* __restrict__ R, long long dim,
                           int nb) {
    long long total = (long long)nb * dim;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int k = (int)(e / dim);
        R[e] = AX[e] - theta[k] * X[e];
    }
}

// D[k] = R[sel[k]] / (theta[sel[k]] - diag)   (|theta - diag| floored at 1e-8)
__global__ void k_precond(const double* __restrict__ R, const double* __restrict__ diag,
                          const double* __restrict__ theta, const int* __restrict__ sel,
                          double* __restrict__ D, long long dim, int nsel) {
    long long total = (long long)nsel * dim;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int k = (int)(e / dim);
        long long x = e - (long long)k * dim;
        int r = sel[k];
        double den = theta[r] - diag[x];
        if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
        D[e] = R[(long long)r * dim + x] / den;
    }
}

__global__ void k_scale(double* x, double a, long long n) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        x[e] *= a;
}

__global__ void k_unit(double* V, const long long* idx, long long dim, int nb) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nb) V[(long long)k * dim + idx[k]] = 1.0;
}

static unsigned nb_(long long n) {
    long long g = (n + 255) / 256;
    if (g > (1LL << 20)) g = 1LL << 20;
    return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
struct Dav {
    adc_ctx* c;
    Engine& E;
    long long dim;
    int block, max_space;
    DBuf<double> V, W, X, AX, R, D, G, S, th, ev_e, part, rn, cmat, tmp, gb;
    DBuf<int> sel_d, info;
    int nchunk = 0;

    explicit Dav(adc_ctx* cc) : c(cc), E(cc->E), dim(cc->dim) {}

    void rownorms(const double* M, int nrow, std::vector<double>& out) {
        nchunk = (int)std::min<long long>(256, (dim + 4095) / 4096);
        if (nchunk < 1) nchunk = 1;
        part.ensure((size_t)nrow * nchunk, &c->arena);
        rn.ensure(nrow, &c->arena);
        hipLaunchKernelGGL(k_rownorm_part, dim3(nchunk, nrow), dim3(256), 0, E.stream, M, dim,
                           nchunk, part.p);
        hipLaunchKernelGGL(k_rownorm_final, dim3((nrow + 63) / 64), dim3(64), 0, E.stream, part.p,
                           nchunk, nrow, rn.p);
        ADC_HIP(hipGetLastError());
        out.resize(nrow);
        ADC_HIP(hipMemcpyAsync(out.data(), rn.p, nrow * sizeof(double), hipMemcpyDeviceToHost,
                               E.stream));
        ADC_HIP(hipStreamSynchronize(E.stream));
    }

    // orthonormalise nd rows of Dm against V[0:m] and among themselves.  One
    // pass, or two when the first shrank a direction below 1e-3 of its norm,
    // of: block classical Gram-Schmidt against V, twice (one long-K GEMM each
    // way), then the block's own Gram matrix G = Dm Dm^T, diagonalised on the
    // host (nd is small), and Dm <- L^-1/2 U^T Dm over the eigenpairs with
    // lambda > max(1e-20, 1e-14 lambda_max): directions that fall below (rows
    // of unit norm that are numerically dependent on V or on each other) are
    // dropped.  The kept rows are compacted to the front; returns their count.
    int orthonormalize(double* Dm, int nd, int m) {
        cmat.ensure((size_t)std::max(1, nd * std::max(m, nd)), &c->arena);
        std::vector<double> nrm;
        rownorms(Dm, nd, nrm);
        for (int k = 0; k < nd; ++k) {
            double s = (nrm[k] > 0 && std::isfinite(nrm[k])) ? 1.0 / nrm[k] : 0.0;
            hipLaunchKernelGGL(k_scale, dim3(nb_(dim)), dim3(256), 0, E.stream,
                               Dm + (size_t)k * dim, s, dim);
        }
        ADC_HIP(hipGetLastError());
        tmp.ensure((size_t)nd * dim, &c->arena);
        std::vector<double> G, T;
        bool last = false;
        for (int pass = 0; pass < 2 && nd > 0 && !last; ++pass) {
            if (m > 0) {
                for (int cgs = 0; cgs < 2; ++cgs) {
                    gemm_rm<double>(E, false, true, nd, m, dim, 1.0, Dm, dim, 0, V.p, dim, 0, 0.0,
                                    cmat.p, m, 0, 1);
                    gemm_rm<double>(E, false, false, nd, dim, m, -1.0, cmat.p, m, 0, V.p, dim, 0,
                                    1.0, Dm, dim, 0, 1);
                }
            }
            gemm_rm<double>(E, false, true, nd, nd, dim, 1.0, Dm, dim, 0, Dm, dim, 0, 0.0, cmat.p,
                            nd, 0, 1);
            G.resize((size_t)nd * nd);
            ADC_HIP(hipMemcpyAsync(G.data(), cmat.p, G.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, E.stream));
            ADC_HIP(hipStreamSynchronize(E.stream));
            for (int i = 0; i < nd; ++i)
                for (int j = 0; j < i; ++j) {
                    double v = 0.5 * (G[(size_t)i * nd + j] + G[(size_t)j * nd + i]);
                    G[(size_t)i * nd + j] = G[(size_t)j * nd + i] = v;
                }
            std::vector<double> lam, U;
            jacobi_eigen(G, nd, lam, U);
            double lmax = 0.0;
            for (double l : lam) lmax = std::max(lmax, l);
            const double cut = std::max(1e-20, 1e-14 * lmax);
            T.clear();
            int kept = 0;
            double lmin_kept = INFINITY;
            for (int k = 0; k < nd; ++k) {
                if (!(lam[k] > cut) || !std::isfinite(lam[k])) continue;
                const double f = 1.0 / std::sqrt(lam[k]);
                for (int j = 0; j < nd; ++j) T.push_back(U[(size_t)j * nd + k] * f);
                ++kept;
                lmin_kept = std::min(lmin_kept, lam[k]);
            }
            if (kept == 0) return 0;
            // the second pass only when the first left directions of small
            // norm (unit rows shrunk below 1e-3 by the projections or among
            // themselves): scaling them back up by 1/sqrt(lambda) would also
            // scale their remaining components along V
            if (pass == 0 && lmin_kept >= 1e-6) last = true;
            ADC_HIP(hipMemcpyAsync(cmat.p, T.data(), T.size() * sizeof(double),
                                   hipMemcpyHostToDevice, E.stream));
            gemm_rm<double>(E, false, false, kept, dim, nd, 1.0, cmat.p, nd, 0, Dm, dim, 0, 0.0,
                            tmp.p, dim, 0, 1);
            ADC_HIP(hipMemcpyAsync(Dm, tmp.p, (size_t)kept * dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, E.stream));
            nd = kept;
        }
        ADC_HIP(hipStreamSynchronize(E.stream));
        return nd;
    }

    // eigenpairs of a small symmetric matrix (cyclic Jacobi rotations):
    // lam[k], U[j][k] = component j of eigenvector k
    static void jacobi_eigen(std::vector<double> A, int n, std::vector<double>& lam,
                             std::vector<double>& U) {
        U.assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
        for (int sweep = 0; sweep < 100; ++sweep) {
            double off = 0.0, diag = 0.0;
            for (int i = 0; i < n; ++i) {
                diag += A[(size_t)i * n + i] * A[(size_t)i * n + i];
                for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
            }
            if (off <= 1e-32 * diag || off == 0.0) break;
            for (int p = 0; p < n; ++p)
                for (int q = p + 1; q < n; ++q) {
                    const double apq = A[(size_t)p * n + q];
                    if (apq == 0.0) continue;
                    const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                    const double th = 0.5 * (aqq - app) / apq;
                    const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                    const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                    for (int k = 0; k < n; ++k) {
                        const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                        A[(size_t)k * n + p] = cs * akp - sn * akq;
                        A[(size_t)k * n + q] = sn * akp + cs * akq;
                    }
                    for (int k = 0; k < n; ++k) {
                        const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                        A[(size_t)p * n + k] = cs * apk - sn * aqk;
                        A[(size_t)q * n + k] = sn * apk + cs * aqk;
                    }
                    for (int k = 0; k < n; ++k) {
                        const double ukp = U[(size_t)k * n + p], ukq = U[(size_t)k * n + q];
                        U[(size_t)k * n + p] = cs * ukp - sn * ukq;
                        U[(size_t)k * n + q] = sn * ukp + cs * ukq;
                    }
                }
        }
        lam.resize(n);
        for (int i = 0; i < n; ++i) lam[i] = A[(size_t)i * n + i];
    }
};

// One solve as a state machine, so that several systems can advance in
// lockstep with their sigma products batched (batch.hip):
//   Solver s(c, nroots);  while (s.request(&X, &W, &n, &prec)) { sigma; s.advance(); }
//   s.finish(energies, P, vecs, n_iter);
struct Solver {
    using clk = std::chrono::steady_clock;
    adc_ctx* c;
    Engine& E;
    int nroots;
    long long dim;
    int block, max_space;
    double tol_e, tol_r, tol_switch, tol_switch2;
    const double rel_switch = 3e-3;
    Dav d;
    clk::time_point t0;
    std::vector<double> theta_old, theta, rnorm, Gh, blk, Sh;
    int it = 0, status = ADC_OK, m = 0, newstart = 0, nbk = 0;
    int stage = 0;    // sigma level of the current phase: 1 BF16, 2 FP32 products, 0 FP64
    bool use_mlp, done = false;
    double best_mixed_r = INFINITY, best_mlp_r = INFINITY;
    int stall = 0, mlp_stall = 0;
    // wall seconds per phase (verbose >= 2): sigma (timed by the driver), the
    // new rows of V W^T, eigenpairs + Ritz vectors + residuals, the rest
    double ph[4] = {0, 0, 0, 0};
    clk::time_point tp;
    void lap(int k) {
        const auto now = clk::now();
        ph[k] += std::chrono::duration<double>(now - tp).count();
        tp = now;
    }

    Solver(adc_ctx* cc, int nr) : c(cc), E(cc->E), nroots(nr), dim(cc->dim), d(cc) {
        t0 = clk::now();
        block = c->block > 0 ? c->block : std::max(nroots, 8);
        block = std::max(block, nroots);
        block = (int)std::min<long long>(block, dim);
        max_space = c->max_space > 0 ? c->max_space : 8 * block;
        if (c->max_space <= 0) {
            // default bound: V and W within a quarter of the free device memory
            // (large systems), but room for three blocks of vectors
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
                const long long fit = (long long)(fr / 4 / (2 * sizeof(double) * (size_t)dim));
                max_space = (int)std::max<long long>(3LL * block, std::min<long long>(max_space, fit));
            } else {
                (void)hipGetLastError();
            }
        }
        max_space = std::max(max_space, 2 * block);
        max_space = (int)std::min<long long>(max_space, dim);
        tol_e = c->tol_e;
        tol_r = c->tol_r > 0 ? c->tol_r : std::sqrt(tol_e);
        // leave the reduced-precision phase once the residuals reach what BF16
        // products can resolve, or when they stop falling
        tol_switch = std::max(std::sqrt(tol_r), 1e-3);
        // and the FP32-product phase at what FP32 sums resolve
        tol_switch2 = std::max(tol_r, 2e-6);
        d.block = block;
        d.max_space = max_space;
        d.V.alloc((size_t)max_space * dim, &c->arena);
        d.W.alloc((size_t)max_space * dim, &c->arena);
        d.X.alloc((size_t)block * dim, &c->arena);
        d.AX.alloc((size_t)block * dim, &c->arena);
        d.R.alloc((size_t)block * dim, &c->arena);
        d.D.alloc((size_t)block * dim, &c->arena);
        d.G.alloc((size_t)max_space * max_space, &c->arena);
        d.S.alloc((size_t)max_space * max_space, &c->arena);
        d.th.alloc(max_space, &c->arena);
        d.ev_e.alloc(max_space, &c->arena);
        d.sel_d.alloc(block, &c->arena);
        d.info.alloc(2, &c->arena);   // status, Jacobi sweeps
        initial_space();
        theta_old.assign(block, INFINITY);
        theta.assign(max_space, 0.0);
        Gh.assign((size_t)max_space * max_space, 0.0);
        stage = c->precision >= 1 ? 1 : 0;
        use_mlp = c->use_mlp && c->mlp_params.p;
        c->st_sigvec = 0;
        c->st_mixed = 0;
        c->hist_nroots = nroots;
        c->hist_t.clear();
        c->hist_theta.clear();
        c->hist_r.clear();
        c->hist_mixed.clear();
        // iterates recorded for training pairs
        c->nrec = 0;
        c->rec_theta.clear();
        c->rec_root.clear();
        if (c->record_max > 0) {
            c->rec_x.alloc((size_t)c->record_max * dim, &c->arena);
            c->rec_r.alloc((size_t)c->record_max * dim, &c->arena);
        }
    }

    void initial_space() {
        int nb = 0;
        if (c->nguess > 0) {
            nb = std::min(c->nguess, block);
            ADC_HIP(hipMemcpyAsync(d.V.p, c->guess.p, (size_t)nb * dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, E.stream));
            nb = d.orthonormalize(d.V.p, nb, 0);
        }
        if (nb < block) {
            std::vector<double> dh(dim);
            ADC_HIP(hipMemcpyAsync(dh.data(), c->diag.p, dim * sizeof(double),
                                   hipMemcpyDeviceToHost, E.stream));
            ADC_HIP(hipStreamSynchronize(E.stream));
            std::vector<long long> ord(dim);
            std::iota(ord.begin(), ord.end(), 0LL);
            int need = block - nb;
            std::partial_sort(ord.begin(), ord.begin() + std::min<long long>(dim, need + nb),
                              ord.end(), [&](long long a, long long b) {
                                  return dh[a] < dh[b] || (dh[a] == dh[b] && a < b);
                              });
            // unit vectors, orthogonalised against any guess vectors
            double* Dm = d.V.p + (size_t)nb * dim;
            fill<double>(E, Dm, 0.0, (size_t)need * dim);
            DBuf<long long> idx;
            idx.alloc(need, &c->arena);
            ADC_HIP(hipMemcpyAsync(idx.p, ord.data(), need * sizeof(long long),
                                   hipMemcpyHostToDevice, E.stream));
            hipLaunchKernelGGL(k_unit, dim3((need + 63) / 64), dim3(64), 0, E.stream, Dm, idx.p,
                               dim, need);
            ADC_HIP(hipGetLastError());
            ADC_HIP(hipStreamSynchronize(E.stream));
            if (nb > 0) {
                int kept = d.orthonormalize(Dm, need, nb);
                nb += kept;
            } else {
                nb = need;
            }
        }
        m = nb;
        newstart = 0;
        if (m < nroots)
            throw Error(ADC_E_NUMERIC, "initial Davidson space: " + std::to_string(m) +
                                           " independent vectors for " + std::to_string(nroots) +
                                           " roots (dependent guess vectors?)");
    }

    // sigma work of the coming iteration: the basis vectors without a sigma
    // vector.  Returns false once the solve has ended.
    bool request(const double** X, double** W, int* nn, int* precision) {
        if (done) return false;
        if (c->verbose >= 2) {
            ADC_HIP(hipStreamSynchronize(E.stream));
            tp = clk::now();
        }
        *X = d.V.p + (size_t)newstart * dim;
        *W = d.W.p + (size_t)newstart * dim;
        *nn = m - newstart;
        *precision = stage;
        return true;
    }

    // everything after the sigma products; returns true when the solve ended
    bool advance() {
        if (c->verbose >= 2) {
            ADC_HIP(hipStreamSynchronize(E.stream));
            lap(0);
        }
        ++it;
        const int nn = m - newstart;
        c->st_sigvec += nn;
        if (stage) c->st_mixed++;
        // G rows for the new vectors: blk[nn][m] = W_new V^T
        {
            DBuf<double>& gb = d.gb;
            gb.ensure((size_t)nn * m, &c->arena);
            gemm_rm<double>(E, false, true, nn, m, dim, 1.0, d.W.p + (size_t)newstart * dim, dim, 0,
                            d.V.p, dim, 0, 0.0, gb.p, m, 0, 1);
            blk.resize((size_t)nn * m);
            ADC_HIP(hipMemcpyAsync(blk.data(), gb.p, blk.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, E.stream));
            ADC_HIP(hipStreamSynchronize(E.stream));
            if (c->verbose >= 2) lap(1);
            for (int k = 0; k < nn; ++k) {
                const int r = newstart + k;
                for (int j = 0; j < newstart; ++j) {
                    double v = blk[(size_t)k * m + j];
                    Gh[(size_t)r * max_space + j] = v;
                    Gh[(size_t)j * max_space + r] = v;
                }
                for (int j2 = 0; j2 < nn; ++j2) {
                    const int j = newstart + j2;
                    Gh[(size_t)r * max_space + j] =
                        0.5 * (blk[(size_t)k * m + j] + blk[(size_t)j2 * m + r]);
                }
            }
        }
        newstart = m;
        // projected eigenproblem: on the host (the matrix is there already), or by
        // rocSOLVER (column-major == row-major for symmetric input)
        std::vector<double> Gc((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Gc[(size_t)i * m + j] = Gh[(size_t)i * max_space + j];
        const bool on_host = c->eigensolver == 2 || (c->eigensolver == 0 && m <= 64);
        Sh.resize((size_t)m * m);
        // (rocSOLVER takes over should the host QR sweeps not converge)
        if (on_host && syev_host(m, Gc.data(), theta.data(), Sh.data(), std::min(block, m))) {
            ADC_HIP(hipMemcpyAsync(d.S.p, Sh.data(), Sh.size() * sizeof(double),
                                   hipMemcpyHostToDevice, E.stream));
            ADC_HIP(hipMemcpyAsync(d.th.p, theta.data(), m * sizeof(double),
                                   hipMemcpyHostToDevice, E.stream));
        } else {
            ADC_HIP(hipMemcpyAsync(d.S.p, Gc.data(), Gc.size() * sizeof(double),
                                   hipMemcpyHostToDevice, E.stream));
            if (c->eigensolver == 1)
                ADC_BLAS(rocsolver_dsyevj(E.blas, rocblas_esort_ascending, rocblas_evect_original,
                                          rocblas_fill_upper, m, d.S.p, m, 0.0, d.ev_e.p, 100,
                                          d.info.p + 1, d.th.p, d.info.p));
            else
                ADC_BLAS(rocsolver_dsyevd(E.blas, rocblas_evect_original, rocblas_fill_upper, m,
                                          d.S.p, m, d.th.p, d.ev_e.p, d.info.p));
            ADC_HIP(hipMemcpyAsync(theta.data(), d.th.p, m * sizeof(double),
                                   hipMemcpyDeviceToHost, E.stream));
            int info = 0;
            ADC_HIP(hipMemcpyAsync(&info, d.info.p, sizeof(int), hipMemcpyDeviceToHost,
                                   E.stream));
            ADC_HIP(hipStreamSynchronize(E.stream));
            if (info != 0)
                throw Error(ADC_E_NUMERIC, "projected eigenproblem: rocSOLVER did not converge "
                                           "(info " + std::to_string(info) + ")");
        }
        nbk = std::min(block, m);
        if (nbk < nroots)
            throw Error(ADC_E_NUMERIC, "Davidson basis holds " + std::to_string(m) +
                                           " independent vectors, fewer than the " +
                                           std::to_string(nroots) + " roots asked for");
        // Ritz vectors: X = S^T V, AX = S^T W  (row k of S is eigenvector k)
        gemm_rm<double>(E, false, false, nbk, dim, m, 1.0, d.S.p, m, 0, d.V.p, dim, 0, 0.0, d.X.p,
                        dim, 0, 1);
        gemm_rm<double>(E, false, false, nbk, dim, m, 1.0, d.S.p, m, 0, d.W.p, dim, 0, 0.0,
                        d.AX.p, dim, 0, 1);
        hipLaunchKernelGGL(k_residual, dim3(nb_((long long)nbk * dim)), dim3(256), 0, E.stream,
                           d.AX.p, d.X.p, d.th.p, d.R.p, dim, nbk);
        ADC_HIP(hipGetLastError());
        d.rownorms(d.R.p, nbk, rnorm);
        if (c->verbose >= 2) lap(2);
        for (int k = 0; k < nbk; ++k)
            if (!std::isfinite(rnorm[k]) || !std::isfinite(theta[k]))
                throw Error(ADC_E_NUMERIC, "non-finite Ritz value or residual");
        c->hist_t.push_back(std::chrono::duration<double>(clk::now() - t0).count());
        for (int k = 0; k < nroots; ++k) {
            c->hist_theta.push_back(k < nbk ? theta[k] : NAN);
            c->hist_r.push_back(k < nbk ? rnorm[k] : NAN);
        }
        c->hist_mixed.push_back(stage);
        for (int k = 0; k < nroots && k < nbk && c->nrec < c->record_max; ++k) {
            ADC_HIP(hipMemcpyAsync(c->rec_x.p + (size_t)c->nrec * dim, d.X.p + (size_t)k * dim,
                                   dim * sizeof(double), hipMemcpyDeviceToDevice, E.stream));
            ADC_HIP(hipMemcpyAsync(c->rec_r.p + (size_t)c->nrec * dim, d.R.p + (size_t)k * dim,
                                   dim * sizeof(double), hipMemcpyDeviceToDevice, E.stream));
            c->rec_theta.push_back(theta[k]);
            c->rec_root.push_back(k);
            ++c->nrec;
        }
        // residuals in units of max(1, |theta|): relative for large roots;
        // eigenvalue changes against tol_e, or against the FP64 resolution of
        // theta (8 ulp) where that is coarser: changes below it are rounding
        double maxde = 0.0, maxr = 0.0;
        bool e_ok = true;
        for (int k = 0; k < nroots; ++k) {
            const double de = std::fabs(theta[k] - theta_old[k]);
            maxde = std::max(maxde, de);
            e_ok = e_ok && de <= std::max(tol_e, 8.0 * DBL_EPSILON * std::fabs(theta[k]));
            maxr = std::max(maxr, rnorm[k] / std::max(1.0, std::fabs(theta[k])));
        }
        if (c->verbose) {
            fprintf(stderr, "adc_davidson it %d %.2f s m %d nbk %d %s max|dE| %.3e max|r| %.3e theta:",
                    it, c->hist_t.back(), m, nbk, stage == 1 ? "bf16" : stage == 2 ? "fp32" : "fp64",
                    maxde, maxr);
            for (int k = 0; k < nbk; ++k) fprintf(stderr, " %.10f(%.1e)", theta[k], rnorm[k]);
            fprintf(stderr, "\n");
        }
        if (stage) {
            // stagnation: three iterations in a row without a 10% decrease
            // (ordinary convergence shrinks residuals by 2-3x per iteration;
            // a reduced-precision sigma stalls at its rounding level)
            stall = (maxr > 0.9 * best_mixed_r) ? stall + 1 : 0;
            best_mixed_r = std::min(best_mixed_r, maxr);
        }
        const double sw = stage == 1 ? tol_switch : tol_switch2;
        if (stage && (maxr <= sw || (stage == 1 && maxr <= rel_switch) || stall >= 3)) {
            // refinement: the next level (FP32 products after BF16 when asked
            // for, then FP64) rebuilds the space from the Ritz vectors
            stage = (stage == 1 && c->precision == 2) ? 2 : 0;
            if (stage == 0) release_mixed(c);   // room for the FP64 products
            stall = 0;
            best_mixed_r = INFINITY;
            ADC_HIP(hipMemcpyAsync(d.V.p, d.X.p, (size_t)nbk * dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, E.stream));
            m = d.orthonormalize(d.V.p, nbk, 0);
            newstart = 0;
            std::fill(Gh.begin(), Gh.end(), 0.0);
            std::fill(theta_old.begin(), theta_old.end(), INFINITY);
            return false;
        }
        if (!stage && e_ok && maxr <= tol_r) return end(ADC_OK);
        if (it >= c->max_iter) return end(ADC_E_NOCONV);
        for (int k = 0; k < nbk; ++k) theta_old[k] = theta[k];
        std::vector<int> sel;
        double thr = stage == 1 ? tol_switch : stage == 2 ? tol_switch2 : tol_r;
        for (int k = 0; k < nbk; ++k)
            if (rnorm[k] > thr * std::max(1.0, std::fabs(theta[k]))) sel.push_back(k);
        if (sel.empty())
            for (int k = 0; k < nroots; ++k) sel.push_back(k);
        int nsel = (int)sel.size();
        // learned correction of the diagonal preconditioner while it behaves:
        // a non-finite output, or residuals that stop falling (four
        // iterations without a 10% decrease), switch to the diagonal one
        if (use_mlp) {
            mlp_stall = (maxr > 0.9 * best_mlp_r) ? mlp_stall + 1 : 0;
            best_mlp_r = std::min(best_mlp_r, maxr);
            if (mlp_stall >= 4) use_mlp = false;
        }
        bool precond_done = false;
        if (use_mlp) {
            precond_done = mlp_precondition(c, d.R.p, theta, sel, d.D.p);
            if (!precond_done) use_mlp = false;
        }
        if (!precond_done) {
            ADC_HIP(hipMemcpyAsync(d.sel_d.p, sel.data(), nsel * sizeof(int),
                                   hipMemcpyHostToDevice, E.stream));
            hipLaunchKernelGGL(k_precond, dim3(nb_((long long)nsel * dim)), dim3(256), 0,
                               E.stream, d.R.p, c->diag.p, d.th.p, d.sel_d.p, d.D.p, dim, nsel);
            ADC_HIP(hipGetLastError());
        }
        if (m + nsel > max_space) {
            // restart from the current Ritz vectors
            ADC_HIP(hipMemcpyAsync(d.V.p, d.X.p, (size_t)nbk * dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, E.stream));
            ADC_HIP(hipMemcpyAsync(d.W.p, d.AX.p, (size_t)nbk * dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, E.stream));
            std::fill(Gh.begin(), Gh.end(), 0.0);
            for (int k = 0; k < nbk; ++k) Gh[(size_t)k * max_space + k] = theta[k];
            m = nbk;
            newstart = m;
        }
        int kept = d.orthonormalize(d.D.p, nsel, m);
        if (kept == 0) {
            // every correction lies in the current space: the space is invariant
            // to working precision, so the Ritz pairs are converged if their
            // residuals are
            return end((!stage && maxr <= tol_r) ? ADC_OK : ADC_E_NOCONV);
        }
        ADC_HIP(hipMemcpyAsync(d.V.p + (size_t)m * dim, d.D.p,
                               (size_t)kept * dim * sizeof(double), hipMemcpyDeviceToDevice,
                               E.stream));
        m += kept;
        if (c->verbose >= 2) lap(3);
        return false;
    }

    bool end(int st) {
        status = st;
        done = true;
        return true;
    }

    int finish(double* energies, double* P, double* vecs, int* n_iter) {
        if (c->verbose >= 2 && it > 0)
            fprintf(stderr, "adc_davidson phases per iteration (ms): sigma %.3f, V W^T rows %.3f, "
                    "eigenpairs+Ritz+residuals %.3f, preconditioner+orthonormalisation %.3f\n",
                    1e3 * ph[0] / it, 1e3 * ph[1] / it, 1e3 * ph[2] / it, 1e3 * ph[3] / it);
        if (c->use_mlp && !use_mlp) c->mlp_fallbacks++;
        for (int k = 0; k < nroots; ++k) energies[k] = theta[k];
        if (vecs)
            ADC_HIP(hipMemcpyAsync(vecs, d.X.p, (size_t)nroots * dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, E.stream));
        if (P) {
            DBuf<double> Xs;
            Xs.alloc((size_t)nroots * c->nspec(), &c->arena);
            spec_amplitudes(c, d.X.p, nroots, Xs.p);
            std::vector<double> xh((size_t)nroots * c->nspec());
            ADC_HIP(hipMemcpyAsync(xh.data(), Xs.p, xh.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, E.stream));
            ADC_HIP(hipStreamSynchronize(E.stream));
            for (int k = 0; k < nroots; ++k) {
                double s = 0.0;
                for (int p = 0; p < c->nspec(); ++p)
                    s += xh[(size_t)k * c->nspec() + p] * xh[(size_t)k * c->nspec() + p];
                P[k] = c->spec_scale() * s;
            }
        }
        ADC_HIP(hipStreamSynchronize(E.stream));
        if (n_iter) *n_iter = it;
        c->st_iters = it;
        c->st_seconds = std::chrono::duration<double>(clk::now() - t0).count();
        E.scratch.clear();    // also invalidates captured sigma graphs
        return status;
    }
};

Solver* solver_new(adc_ctx* c, int nroots) { return new Solver(c, nroots); }
void solver_delete(Solver* s) { delete s; }
bool solver_request(Solver* s, const double** X, double** W, int* nn, int* precision) {
    return s->request(X, W, nn, precision);
}
bool solver_advance(Solver* s) { return s->advance(); }
int solver_finish(Solver* s, double* energies, double* P, double* vecs, int* n_iter) {
    return s->finish(energies, P, vecs, n_iter);
}

int davidson(adc_ctx* c, int nroots, double* energies, double* P, double* vecs, int* n_iter) {
    Solver s(c, nroots);
    const double* X;
    double* W;
    int nn, precision;
    while (s.request(&X, &W, &nn, &precision)) {
        sigma(c, X, W, nn, precision);
        s.advance();
    }
    return s.finish(energies, P, vecs, n_iter);
}

}  // namespace adc
