// The library context: sizes, options, resident device tensors.
#pragma once

#include "adc_internal.hpp"
#include "mfma_gemm.hpp"

#include <chrono>

struct adc_ctx {
    // sizes
    int O = 0, V = 0, Q = 0, N = 0, order = 2, kind = ADC_EA;
    long long dim = 0;     // ADC matrix dimension
    int n1 = 0;            // 1p (EA: V) or 1h (IP: O) block size
    long long n2x = 0;     // leading extent of the 2p1h/2h1p block (EA: O, IP: V)
    long long n2p = 0;     // pair extent (EA: V, IP: O)

    // options
    int precision = 0;     // 0 fp64, 1 mixed
    int block = 0;         // 0: automatic
    int max_space = 0;     // 0: automatic
    int max_iter = 300;
    double tol_e = 1e-8;
    double tol_r = -1.0;   // <0: sqrt(tol_e)
    int verbose = 0;
    int eigensolver = 0;   // projected eigenproblem: 0 auto, 1 Jacobi, 2 host QR, 3 divide and conquer

    adc::Arena arena;
    adc::Engine E;
    hipStream_t user_stream = nullptr;
    bool own_blas = false;

    // resident FP64 tensors (layouts in setup.hip)
    adc::DBuf<double> eo, ev;
    adc::DBuf<double> Boo, Bov, Bvv, Bvo;
    adc::DBuf<double> ovov, oovv, ooov, oooo;
    adc::DBuf<double> t, s, u, w;       // amplitudes
    adc::DBuf<double> M11;              // [n1][n1]
    adc::DBuf<double> gam;              // ADC(3) coupling intermediate [O][V] (EA: [j][b], IP: [j][b])
    adc::DBuf<double> diag;             // [dim]
    adc::DBuf<double> rho, om, ttu;     // spectroscopic-amplitude helpers
    adc::DBuf<double> tt;               // t~ = 2 t_ij^ab - t_ij^ba (order 3)
    adc::DBuf<double> Om, Pi;           // IP-ADC(3) precontracted blocks [O][O][O][V]
    // 1p-1p / 1h-1h block applied on the fly (setup option "m11_onthefly",
    // m11_fly.hip): M11 then holds only its diagonal through second order, and
    // the intermediates below stay resident (u also stays for order 3)
    bool m11_fly = false;
    adc::DBuf<double> Du, Lam, P, P7, Pt, wq;   // D u, Lambda, P_kl, P7_ijkl, Pt_ce, Pt.(ce|Q)
    // unrestricted (open-shell) reference, uadc.hip: O, V above are the alpha
    // counts; the spin blocks live here
    bool uhf = false;
    struct Uhf {
        int Oa = 0, Ob = 0, Va = 0, Vb = 0;
        long long off[7] = {0, 0, 0, 0, 0, 0, 0};   // Y1a Y1b aaa bab aab bbb | end
        adc::DBuf<double> eoa, eva, eob, evb;
        adc::DBuf<double> Booa, Bova, Bvva, Boob, Bovb, Bvvb;
        adc::DBuf<double> taa, tab, tbb, t1a, t1b, M11a, M11b, rhoa, rhob;
    } uh;
    // spectroscopic amplitudes per vector: N spatial orbitals (closed shell,
    // Eq. 50 carries the factor 2 of the two spins) or 2N spin orbitals
    int nspec() const { return uhf ? 2 * N : N; }
    double spec_scale() const { return uhf ? 1.0 : 2.0; }
    adc::DBuf<double> guess;            // warm start
    int nguess = 0;

    // mixed-precision copies of the sigma operands (FP32; B_vv also as BF16
    // for the particle-particle rebuild), made on first use
    adc::DBuf<float> fBoo, fBov, fBvo, fBvv, fM11, fovov, foovv, fooov, foooo, ft, ftt, fgam, fOm,
        fPi;
    adc::DBuf<adc::bf16_t> hBvv;
    bool mixed_ready = false;

    // EA sigma operands rearranged so that every large contraction is one
    // product with both summed index runs contiguous (ea_layout.hip); made on
    // the first EA-ADC(3) sigma of each precision when they fit in memory
    int ea_layout = -1;   // option: -1 automatic, 0 generic contraction path, 1 arranged
    struct EaLayout {
        // FP64: ttT1[k][d][j][c] = t~_jk^cd, ttT2[k][d][j][c] = t~_jk^dc,
        // tT1[k][d][j][c] = t_jk^cd, tD[i][a][k][d] = t_ik^da,
        // oovvT[i][b][j][c] = (ji|bc), tT[a][b][k][l] = t_kl^ab,
        // G[a][j][k][l] = (jk|la) - 2 (jl|ka);
        // H[i][b][Q] = sum_kd t~_ik^bd B^Q_kd and BH = B_ov + H (folded coupling operands)
        adc::DBuf<double> ttT1, ttT2, tT1, tD, oovvT, tT, G, H, BH;
        // mixed: BF16 copies of the product operands (rounded through FP32,
        // as the FP32 copies are when staged) and FP32 G
        adc::DBuf<adc::bf16_t> httT1, httT2, htT1, htD, hoovvT, htT, hovov;
        adc::DBuf<float> fG, fH, fBH;
        // FP32 copies for the FP32-product level
        adc::DBuf<float> fttT1, fttT2, ftT1, ftD, foovvT, ftT;
        bool ready = false, ready_mixed = false, ready_f32 = false;
        // the current call's path: 1 arranged operands resident, 2 built per
        // call in blocks from t, (ov|ov) and (oo|vv) (option value 2, or the
        // automatic choice when the resident ones do not fit)
        int mode = 0;
        bool ready_blocked = false;
    } eal;
    // t~ + u~ parked in pinned host memory (the blocked EA path frees device
    // memory for large systems); the spectroscopic amplitudes stream it back
    double* ttu_host = nullptr;
    // out-of-core B_vv (option "bvv_host", bvv.hip): the vv block of the DF
    // factors and its FP32 / BF16 copies in pinned host memory
    bool bvv_host = false;
    double* hB64 = nullptr;
    float* hB32 = nullptr;
    adc::bf16_t* hB16 = nullptr;
    bool big_mixed = false;   // FP32 copies of the O^2 V^2 operands made
    long long pp_slab_bytes = 16LL << 30;  // rebuilt four-index slab (particle-particle term)
    bool pp_slab_set = false;              // bound given by option pp_slab_mb
    long long pp_slab_auto = 0;            // default bound chosen from free memory
    int pp_blocks = 0;                     // minimum number of a-blocks of that term (0: automatic)
    int pp_group = 0;                      // blocks per contraction product (0: automatic)

    // sigma replayed from captured HIP graphs (sigma.hip)
    struct SigmaGraph {
        int nvec = 0, precision = 0;
        std::map<int, std::pair<void*, size_t>> slots;   // scratch used by the capture
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    bool use_graph = false;
    hipStream_t gstream = nullptr;   // capture stream when the context runs on the null stream
    hipEvent_t gdone = nullptr;      // marks the end of a replay on gstream
    std::vector<SigmaGraph> graphs;
    adc::DBuf<double> Xg, Yg;     // the captured graphs' input and output
    long long graph_launches = 0;
    long long graph_captures = 0;

    // learned preconditioner (mlp.hip): installed parameters, or diagonal
    double escale = 1.0;                  // max |eps|, the feature energy scale
    adc::DBuf<float> mlp_params;
    bool use_mlp = false;
    int mlp_fallbacks = 0;                // solves that fell back to the diagonal

    // Davidson iterates recorded for training pairs (Ritz vector, residual, value)
    int record_max = 0;
    int nrec = 0;
    adc::DBuf<double> rec_x, rec_r;
    std::vector<double> rec_theta;
    std::vector<int> rec_root;

    // statistics and convergence history of the last solve
    int hist_nroots = 0;
    std::vector<double> hist_t, hist_theta, hist_r;
    std::vector<int> hist_mixed;
    int st_iters = 0, st_mixed = 0;
    long long st_sigvec = 0;
    double st_seconds = 0.0;

    std::string err;

    // setup progress on stderr (adc_set_setup_option "verbose"): one line per
    // phase and per block of the long loops, after synchronising the stream
    int setup_verbose = 0;
    std::chrono::steady_clock::time_point setup_t0;
    void phase(const char* what, long long i = -1, long long n = -1) {
        if (!setup_verbose) return;
        (void)hipStreamSynchronize(E.stream);
        const double s =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - setup_t0).count();
        if (i >= 0)
            fprintf(stderr, "adc_setup %8.1f s  %s %lld/%lld\n", s, what, i, n);
        else
            fprintf(stderr, "adc_setup %8.1f s  %s\n", s, what);
    }
};

namespace adc {

// setup.hip
void setup_all(adc_ctx* c, const double* eps, const double* B);
void build_mixed(adc_ctx* c, bool big = true);   // big: also the O^2 V^2 operands
void ensure_tt(adc_ctx* c);                       // t~ resident again if it was released
void release_mixed(adc_ctx* c);                   // free the FP32 / BF16 copies
void setup_adc3(adc_ctx* c, const double* tt, const double* X1);

// sigma.hip
template <typename T, typename TB>
void sigma_block(adc_ctx* c, const double* X, double* Y, int nvec);

// vvvv.hip: out[x][a][b] = sum_cd (ac|bd) in[x][c][d], (ac|bd) rebuilt from B_vv
// (Bvv null: the rows are staged from the host copy, option "bvv_host").
// npair > 0 declares nx = npair^2 rows x = i npair + j with
// in[(i,j)][c][d] = in[(j,i)][d][c] (the caller guarantees it); the mirrored
// products are then taken from the direct ones instead of being computed.
template <typename T, typename TO>
void vvvv_apply(adc_ctx* c, const T* Bvv, const T* in, TO* out, long long nx, int npair = 0);
void sigma(adc_ctx* c, const double* X, double* Y, int nvec, int precision);
void sigma_eager(adc_ctx* c, const double* X, double* Y, int nvec, int precision);  // one block
void drop_graphs(adc_ctx* c);
// the captured sigma graph of (nvec, precision) when it can be replayed as it
// is (reads Xg, writes Yg), else null
hipGraph_t sigma_graph_ready(adc_ctx* c, int nvec, int precision);
void sigma_cost(const adc_ctx* c, int nvec, double* total, double* pp);

// ea_layout.hip
// level: 0 FP64, 1 BF16 products, 2 FP32 products
bool ea_layout_use(adc_ctx* c, int level);      // arranged EA sigma path for this call?
                                                // (sets eal.mode: 1 resident, 2 blocked)
void ea_layout_build(adc_ctx* c, int level);    // make the arranged operands (once each)
// P1[z][x][j][y] = Y[z][j][x][y], P2[z][x][j][y] = Y[z][j][y][x],
// D = P2 - 2 P1, Pm = 2 P1 - P2 (storage TB), Dw = D (storage T); null outputs skipped
template <typename T, typename TB>
void ea_pairs(Engine& E, const T* Y, int nvec, int O, int V, TB* P1, TB* P2, TB* D, TB* Pm, T* Dw);

// bvv.hip: out-of-core B_vv
void bvv_set_host(adc_ctx* c, bool on);        // move B_vv to pinned host memory or back
void bvv_release_host(adc_ctx* c);             // free the host copies (context teardown)
long long bvv_chunk_rows(const adc_ctx* c, size_t elem);   // rows (a, b) per staged block
// rows [r0, r0 + n) of B_vv (each Q long) in type T, staged into scratch slot `slot`
template <typename T>
const T* bvv_rows(adc_ctx* c, long long r0, long long n, int slot);

// spectrum.hip
void spectral_function(hipStream_t st, const double* w, int nw, const double* e, const double* P,
                       int nr, double eta, double* A);
void propagator_diag(hipStream_t st, const double* w, int nw, const double* e, const double* X,
                     int nr, int norb, double eta, double* G);

// m11_fly.hip: S1 = M11 Y1 (FP64, [nvec][n1]) from the intermediates, without M11
void m11_fly(adc_ctx* c, const double* Y1, double* S1, int nvec);

// spec.hip
void spec_amplitudes(adc_ctx* c, const double* vecs, int nvec,
                     double* Xout /*device [nvec][c->nspec()]*/);

// uadc.hip: unrestricted EA/IP-ADC(2)
void setup_uhf(adc_ctx* c, const double* eps_a, const double* eps_b, const double* B_a,
               const double* B_b);
void sigma_uhf(adc_ctx* c, const double* X, double* Y, int nvec);   // FP64 at every level
void spec_amplitudes_uhf(adc_ctx* c, const double* vecs, int nvec, double* Xout);
void sigma_cost_uhf(const adc_ctx* c, int nvec, double* total);

// mlp.hip: learned preconditioner (layout and features documented there)
constexpr int MLP_NF = 7, MLP_WIDTH = 256;
constexpr long long MLP_NPARAM = MLP_WIDTH * MLP_NF + MLP_WIDTH + MLP_WIDTH * MLP_WIDTH +
                                 MLP_WIDTH + MLP_WIDTH + 1;
void mlp_pairs(adc_ctx* c, const double* x, const double* r, double theta, const double* xstar,
               const long long* idx, long long nidx, float* F, float* a, float* t);
void mlp_forward(adc_ctx* c, const float* P, const float* F, long long n, bool bf16, float* y);
constexpr long long MLP_NOALLOC_ROWS = 8192;   // rows of one no-allocation inference call
void mlp_forward_noalloc(const float* P, const float* F, long long n, bool bf16, float* y,
                         hipStream_t stream);
double mlp_loss_grad(adc_ctx* c, const float* P, const float* F, const float* a, const float* t,
                     long long n, float* G);
void mlp_adam(adc_ctx* c, float* P, const float* G, float* m, float* v, long long np, int step,
              double lr);
bool mlp_precondition(adc_ctx* c, const double* R, const std::vector<double>& theta,
                      const std::vector<int>& sel, double* Dout);

// davidson.hip
int davidson(adc_ctx* c, int nroots, double* energies, double* P, double* vecs, int* n_iter);
// batch.hip: lockstep solves of several systems, sigma of all in one graph launch
struct BatchStats {
    long long graph_launches = 0, captures = 0;
    int iterations = 0;
    long long launches = 0;   // launches of the parent graph (one per iteration at most)
    long long parents = 0;    // parent graphs instantiated
};
int batch_davidson(adc_ctx* const* ctx, int nsys, int nroots, bool use_graph, double* energies,
                   double* P, int* n_iter, int* status, BatchStats* st);
int batch_concurrent(adc_ctx* const* ctx, int nsys, int nroots, bool use_graph, int nthreads,
                     double* energies, double* P, int* n_iter, int* status);
struct Solver;   // one solve as a state machine (batched driving in batch.hip)
Solver* solver_new(adc_ctx* c, int nroots);
void solver_delete(Solver* s);
bool solver_request(Solver* s, const double** X, double** W, int* nn, int* precision);
bool solver_advance(Solver* s);
int solver_finish(Solver* s, double* energies, double* P, double* vecs, int* n_iter);

// kernels shared by setup/sigma (elementwise.hip)
void stage_block(Engine& E, const double* B, int Q, int N, int p0, int np, int q0, int nq,
                 double* out, int Qtot = 0, int Qoff = 0);
// out[p][q][Qoff + Q] = B[Q][p0+p][q0+q] for the Q slices of B (rows of out hold Qtot)
void divide_denom2(Engine& E, double* t, const double* eo, const double* ev, int O, int V,
                   double scale);  // t[i][j][a][b] *= scale / (e_i + e_j - e_a - e_b)
void divide_denom1(Engine& E, double* s, const double* eo, const double* ev, int O, int V,
                   double scale);  // s[i][a] *= scale / (e_i - e_a)
void mul_denom2(Engine& E, const double* t, double* out, const double* eo, const double* ev, int O,
                int V, int i0 = 0, int ni = -1);
// out = (e_a + e_b - e_i - e_j) t on rows i0 .. i0+ni-1 (ni < 0: to the end); t, out
// point at row i0
void mul_denom1(Engine& E, const double* s, double* out, const double* eo, const double* ev, int O,
                int V);            // out = (e_a - e_i) s
template <typename TI, typename TO>
void pair_transform(Engine& E, const TI* in, long long in_stride, long long in_off, TO* out,
                    long long out_stride, long long out_off, int nvec, long long nx, int np,
                    double al, double be, double beta_out);
// out[z][x][p][q] = beta*out + al*in[z][x][p][q] + be*in[z][x][q][p]
template <typename T>
void zeroth_order(Engine& E, const T* Y, T* S, int nvec, long long nx, int np, const double* ex,
                  const double* ep, double sx, double sp);
// S[z][x][p][q] += (sx*ex[x] + sp*(ep[p] + ep[q])) * Y[z][x][p][q]
void symmetrize_m11(Engine& E, double* M, const double* tau, const double* e, int n, double sgn);
// M = sgn*diag(e) - 1/2 (tau + tau^T)
template <typename TI, typename TO>
void copy_rows(Engine& E, const TI* in, long long in_stride, long long in_off, TO* out,
               long long out_stride, long long out_off, int nvec, long long len, double beta_out);
void set_diag(Engine& E, double* d, const double* M11, int n1);
void diag22_adc2(Engine& E, double* d, long long off, long long nx, int np, const double* ex,
                 const double* ep, double sx, double sp);
void diag22_first_order(adc_ctx* c, double* d);

}  // namespace adc
