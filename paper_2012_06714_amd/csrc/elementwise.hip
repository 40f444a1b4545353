// Memory-bound kernels: staging of B, orbital-energy denominators (energies
// staged in LDS), pair transforms of the spin-adapted metric (LDS-tiled
// transposes), zeroth-order sigma and diagonal pieces.
#include "context.hpp"

namespace adc {

static unsigned nblk(long long n, int bs) {
    long long g = (n + bs - 1) / bs;
    if (g > (1LL << 22)) g = 1LL << 22;
    return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// out[p][q][Q] = B[Q][p0+p][q0+q]   (transpose through a 32x33 LDS tile)
// ---------------------------------------------------------------------------
// B holds Q slices (Q <= Qtot); out[r][Qoff + q] with row length Qtot
__global__ void k_stage(const double* __restrict__ B, double* __restrict__ out, int Q, int N, int p0,
                        int np, int q0, int nq, int Qtot, int Qoff) {
    __shared__ double tile[32][33];
    const long long R = (long long)np * nq;
    const long long r0 = (long long)blockIdx.x * 32;
    const int Q0 = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        long long r = r0 + tx;
        int q = Q0 + k;
        double v = 0.0;
        if (r < R && q < Q) {
            long long p = r / nq, qq = r - p * nq;
            v = B[(long long)q * N * N + (p0 + p) * (long long)N + (q0 + qq)];
        }
        tile[k][tx] = v;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        long long r = r0 + k;
        int q = Q0 + tx;
        if (r < R && q < Q) out[r * Qtot + Qoff + q] = tile[tx][k];
    }
}

void stage_block(Engine& E, const double* B, int Q, int N, int p0, int np, int q0, int nq,
                 double* out, int Qtot, int Qoff) {
    if (Qtot <= 0) Qtot = Q;
    long long R = (long long)np * nq;
    ADC_REQUIRE((Q + 31) / 32 <= 65535, "stage_block: too many auxiliary functions per call");
    dim3 grid(nblk(R, 32), (Q + 31) / 32);
    hipLaunchKernelGGL(k_stage, grid, dim3(32, 8), 0, E.stream, B, out, Q, N, p0, np, q0, nq, Qtot,
                       Qoff);
    ADC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// denominators
// ---------------------------------------------------------------------------
// rows i0 .. i0 + ni - 1 of an [i][j][a][b] tensor (t and src point at row i0)
__global__ void k_denom2(double* t, const double* __restrict__ eo, const double* __restrict__ ev,
                         int O, int V, double scale, int mode, const double* __restrict__ src,
                         int i0, int ni) {
    extern __shared__ double sev[];
    for (int a = threadIdx.x; a < V; a += blockDim.x) sev[a] = ev[a];
    __syncthreads();
    const long long VV = (long long)V * V;
    const long long total = (long long)ni * O * VV;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (long long)gridDim.x * blockDim.x) {
        long long ij = x / VV, ab = x - ij * VV;
        int i = i0 + (int)(ij / O), j = (int)(ij - (ij / O) * O);
        int a = (int)(ab / V), b = (int)(ab - (long long)a * V);
        double d = eo[i] + eo[j] - sev[a] - sev[b];
        if (mode == 0)
            t[x] *= scale / d;
        else
            t[x] = -d * src[x];   // (e_a + e_b - e_i - e_j) * src
    }
}

void divide_denom2(Engine& E, double* t, const double* eo, const double* ev, int O, int V,
                   double scale) {
    long long total = (long long)O * O * V * V;
    hipLaunchKernelGGL(k_denom2, dim3(nblk(total, 256)), dim3(256), V * sizeof(double), E.stream, t,
                       eo, ev, O, V, scale, 0, (const double*)nullptr, 0, O);
    ADC_HIP(hipGetLastError());
}

void mul_denom2(Engine& E, const double* t, double* out, const double* eo, const double* ev, int O,
                int V, int i0, int ni) {
    if (ni < 0) ni = O - i0;
    long long total = (long long)ni * O * V * V;
    if (total == 0) return;
    hipLaunchKernelGGL(k_denom2, dim3(nblk(total, 256)), dim3(256), V * sizeof(double), E.stream,
                       out, eo, ev, O, V, 1.0, 1, t, i0, ni);
    ADC_HIP(hipGetLastError());
}

__global__ void k_denom1(double* s, const double* eo, const double* ev, int O, int V, double scale,
                         int mode, const double* src) {
    long long total = (long long)O * V;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (long long)gridDim.x * blockDim.x) {
        int i = (int)(x / V), a = (int)(x - (long long)i * V);
        double d = eo[i] - ev[a];
        if (mode == 0)
            s[x] *= scale / d;
        else
            s[x] = -d * src[x];
    }
}

void divide_denom1(Engine& E, double* s, const double* eo, const double* ev, int O, int V,
                   double scale) {
    hipLaunchKernelGGL(k_denom1, dim3(nblk((long long)O * V, 256)), dim3(256), 0, E.stream, s, eo,
                       ev, O, V, scale, 0, (const double*)nullptr);
    ADC_HIP(hipGetLastError());
}

void mul_denom1(Engine& E, const double* s, double* out, const double* eo, const double* ev, int O,
                int V) {
    hipLaunchKernelGGL(k_denom1, dim3(nblk((long long)O * V, 256)), dim3(256), 0, E.stream, out, eo,
                       ev, O, V, 1.0, 1, s);
    ADC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// pair transform: out[z][x][p][q] = beta*out + al*in[z][x][p][q] + be*in[z][x][q][p]
// one 32x32 (p,q) tile per block; the (q,p) tile is read through LDS so that
// both global reads and the write are coalesced.
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ void k_pair(const TI* __restrict__ in, long long in_stride, long long in_off,
                       TO* __restrict__ out, long long out_stride, long long out_off, long long nzx,
                       long long nx, int np, double al, double be, double beta) {
    __shared__ TI tt[32][33];
    const int tilesq = (np + 31) / 32;
    const int tp = blockIdx.x / tilesq, tq = blockIdx.x - tp * tilesq;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const long long npp = (long long)np * np;
    for (long long zx = blockIdx.y; zx < nzx; zx += gridDim.y) {
        long long z = zx / nx, x = zx - z * nx;
        const TI* src = in + z * in_stride + in_off + x * npp;
        TO* dst = out + z * out_stride + out_off + x * npp;
        // load transposed tile: elements [q][p] for q in tile tq, p in tile tp
        for (int k = ty; k < 32; k += 8) {
            int q = tq * 32 + k, p = tp * 32 + tx;
            tt[k][tx] = (q < np && p < np) ? src[(long long)q * np + p] : TI(0);
        }
        __syncthreads();
        for (int k = ty; k < 32; k += 8) {
            int p = tp * 32 + k, q = tq * 32 + tx;
            if (p < np && q < np) {
                long long o = (long long)p * np + q;
                double v = al * (double)src[o] + be * (double)tt[tx][k];
                if (beta != 0.0) v += beta * (double)dst[o];
                dst[o] = (TO)v;
            }
        }
        __syncthreads();
    }
}

template <typename TI, typename TO>
void pair_transform(Engine& E, const TI* in, long long in_stride, long long in_off, TO* out,
                    long long out_stride, long long out_off, int nvec, long long nx, int np,
                    double al, double be, double beta_out) {
    if (nvec == 0 || nx == 0 || np == 0) return;
    int tiles = (np + 31) / 32;
    long long nzx = (long long)nvec * nx;
    unsigned gy = (unsigned)(nzx < 65535 ? nzx : 65535);
    hipLaunchKernelGGL((k_pair<TI, TO>), dim3(tiles * tiles, gy), dim3(32, 8), 0, E.stream, in,
                       in_stride, in_off, out, out_stride, out_off, nzx, nx, np, al, be, beta_out);
    ADC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// zeroth-order 2p1h / 2h1p sigma: S[z][x][p][q] += (sx ex[x] + sp (ep[p] + ep[q])) Y
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_zeroth(const T* __restrict__ Y, T* __restrict__ S, long long total, long long nx,
                         int np, const double* __restrict__ ex, const double* __restrict__ ep,
                         double sx, double sp) {
    extern __shared__ double sep[];
    for (int p = threadIdx.x; p < np; p += blockDim.x) sep[p] = ep[p];
    __syncthreads();
    const long long npp = (long long)np * np;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        long long zx = e / npp, pq = e - zx * npp;
        long long x = zx % nx;
        int p = (int)(pq / np), q = (int)(pq - (long long)p * np);
        double d = sx * ex[x] + sp * (sep[p] + sep[q]);
        S[e] = (T)((double)S[e] + d * (double)Y[e]);
    }
}

template <typename T>
void zeroth_order(Engine& E, const T* Y, T* S, int nvec, long long nx, int np, const double* ex,
                  const double* ep, double sx, double sp) {
    long long total = (long long)nvec * nx * np * np;
    if (!total) return;
    hipLaunchKernelGGL(k_zeroth<T>, dim3(nblk(total, 256)), dim3(256), np * sizeof(double),
                       E.stream, Y, S, total, nx, np, ex, ep, sx, sp);
    ADC_HIP(hipGetLastError());
}

__global__ void k_diag22(double* d, long long nx, int np, const double* ex, const double* ep,
                         double sx, double sp) {
    const long long npp = (long long)np * np;
    const long long total = nx * npp;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        long long x = e / npp, pq = e - x * npp;
        int p = (int)(pq / np), q = (int)(pq - (long long)p * np);
        d[e] = sx * ex[x] + sp * (ep[p] + ep[q]);
    }
}

void diag22_adc2(Engine& E, double* d, long long off, long long nx, int np, const double* ex,
                 const double* ep, double sx, double sp) {
    long long total = nx * np * np;
    hipLaunchKernelGGL(k_diag22, dim3(nblk(total, 256)), dim3(256), 0, E.stream, d + off, nx, np,
                       ex, ep, sx, sp);
    ADC_HIP(hipGetLastError());
}

__global__ void k_m11(double* M, const double* tau, const double* e, int n, double sgn) {
    long long total = (long long)n * n;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < total;
         x += (long long)gridDim.x * blockDim.x) {
        int a = (int)(x / n), b = (int)(x - (long long)a * n);
        double v = -0.5 * (tau[(long long)a * n + b] + tau[(long long)b * n + a]);
        if (a == b) v += sgn * e[a];
        M[x] = v;
    }
}

void symmetrize_m11(Engine& E, double* M, const double* tau, const double* e, int n, double sgn) {
    hipLaunchKernelGGL(k_m11, dim3(nblk((long long)n * n, 256)), dim3(256), 0, E.stream, M, tau, e,
                       n, sgn);
    ADC_HIP(hipGetLastError());
}

__global__ void k_setdiag(double* d, const double* M, int n) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) d[x] = M[(long long)x * n + x];
}

void set_diag(Engine& E, double* d, const double* M11, int n1) {
    hipLaunchKernelGGL(k_setdiag, dim3((n1 + 255) / 256), dim3(256), 0, E.stream, d, M11, n1);
    ADC_HIP(hipGetLastError());
}

template <typename TI, typename TO>
__global__ void k_copy_rows(const TI* __restrict__ in, long long in_stride, long long in_off,
                            TO* __restrict__ out, long long out_stride, long long out_off, int nvec,
                            long long len, double beta) {
    long long total = (long long)nvec * len;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        long long z = e / len, k = e - z * len;
        TO* o = out + z * out_stride + out_off + k;
        double v = (double)in[z * in_stride + in_off + k];
        if (beta != 0.0) v += beta * (double)*o;
        *o = (TO)v;
    }
}

template <typename TI, typename TO>
void copy_rows(Engine& E, const TI* in, long long in_stride, long long in_off, TO* out,
               long long out_stride, long long out_off, int nvec, long long len, double beta_out) {
    long long total = (long long)nvec * len;
    if (!total) return;
    hipLaunchKernelGGL((k_copy_rows<TI, TO>), dim3(nblk(total, 256)), dim3(256), 0, E.stream, in,
                       in_stride, in_off, out, out_stride, out_off, nvec, len, beta_out);
    ADC_HIP(hipGetLastError());
}

#define ADC_PAIR_INST(TI, TO)                                                                  \
    template void pair_transform<TI, TO>(Engine&, const TI*, long long, long long, TO*, long long, \
                                         long long, int, long long, int, double, double, double); \
    template void copy_rows<TI, TO>(Engine&, const TI*, long long, long long, TO*, long long,      \
                                    long long, int, long long, double);
ADC_PAIR_INST(double, double)
ADC_PAIR_INST(float, float)
ADC_PAIR_INST(double, float)
ADC_PAIR_INST(float, double)
ADC_PAIR_INST(double, bf16_t)
ADC_PAIR_INST(bf16_t, bf16_t)
#undef ADC_PAIR_INST
template void zeroth_order<double>(Engine&, const double*, double*, int, long long, int,
                                   const double*, const double*, double, double);
template void zeroth_order<float>(Engine&, const float*, float*, int, long long, int,
                                  const double*, const double*, double, double);

}  // namespace adc

namespace adc {

// ---------------------------------------------------------------------------
// exact diagonal of the first-order 2p1h (EA) / 2h1p (IP) block in the Z basis.
// With M_Y the non-symmetric spin-adapted block and the pair metric
// S = 2 - P_swap, the Z-basis diagonal on a pair p != q is
//   al'^2 H_pq,pq + 2 al' be' H_pq,qp + be'^2 H_qp,qp,   H = S M_Y,
// and on p == q simply M_Y[(pp),(pp)].  d0 = M_Y[(pq x),(pq x)], d1 = M_Y[(pq x),(qp x)].
//   EA (p,q = a,b; x = i):
//     d0 = e_a + e_b - e_i - (ii|bb) + 2 (ib|ib) - (ii|aa) + (aa|bb) - [a=b] (ia|ia)
//     d1 = -(ib|ib) + (ab|ab) + [a=b] (2 (ia|ia) - 2 (ii|aa))
//   IP (p,q = i,j; x = a):
//     d0 = e_a - e_i - e_j + (ii|jj) + 2 (ja|ja) - (jj|aa) - (ii|aa) - [i=j] (ia|ia)
//     d1 = (ij|ij) - (ja|ja) + [i=j] (2 (ia|ia) - 2 (ii|aa))
// Inputs: J[x][p] = (xp|xp) (EA: (ib|ib), IP stores J[a][j] = (ja|ja)),
//         K[x][p] = (xx|pp) (EA: (ii|bb); IP: K[a][j] = (jj|aa)),
//         Dpp[p][q] = (pp|qq), Epp[p][q] = (pq|pq)
// ---------------------------------------------------------------------------
__global__ void k_diag22_first(double* d, long long nx, int np, const double* ex,
                               const double* ep, double sx, double sp, const double* J,
                               const double* K, const double* Dpp, const double* Epp, int ea) {
    const double SQ3 = 1.7320508075688772;
    const double al = 0.5 * (1.0 + 1.0 / SQ3), be = 0.5 * (1.0 - 1.0 / SQ3);
    const long long npp = (long long)np * np;
    const long long total = nx * npp;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        long long x = e / npp, pq = e - x * npp;
        int p = (int)(pq / np), q = (int)(pq - (long long)p * np);
        auto D0 = [&](int u, int v) {
            double z = sx * ex[x] + sp * (ep[u] + ep[v]);
            double r;
            if (ea)
                r = z - K[x * np + v] + 2.0 * J[x * np + v] - K[x * np + u] + Dpp[(long long)u * np + v];
            else
                r = z + Dpp[(long long)u * np + v] + 2.0 * J[x * np + v] - K[x * np + v] - K[x * np + u];
            if (u == v) r -= J[x * np + u];
            return r;
        };
        auto D1 = [&](int u, int v) {
            double r = (ea ? -J[x * np + v] + Epp[(long long)u * np + v]
                           : Epp[(long long)u * np + v] - J[x * np + v]);
            if (u == v) r += 2.0 * J[x * np + u] - 2.0 * K[x * np + u];
            return r;
        };
        double v;
        if (p == q) {
            v = D0(p, p);
        } else {
            double Haa = 2.0 * D0(p, q) - D1(q, p);
            double Hab = 2.0 * D1(p, q) - D0(q, p);
            double Hbb = 2.0 * D0(q, p) - D1(p, q);
            v = al * al * Haa + 2.0 * al * be * Hab + be * be * Hbb;
        }
        d[e] = v;
    }
}

// (pp|qq) and (pq|pq) from B blocks Bpp[p][q][Q]
__global__ void k_pair_ints(const double* Bpp, int np, int Q, double* Dpp, double* Epp) {
    long long total = (long long)np * np;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int p = (int)(e / np), q = (int)(e - (long long)p * np);
        const double* bp = Bpp + ((long long)p * np + p) * Q;
        const double* bq = Bpp + ((long long)q * np + q) * Q;
        const double* bx = Bpp + ((long long)p * np + q) * Q;
        double s = 0.0, s2 = 0.0;
        for (int k = 0; k < Q; ++k) {
            s += bp[k] * bq[k];
            s2 += bx[k] * bx[k];
        }
        Dpp[e] = s;
        Epp[e] = s2;
    }
}

// J[x][p] = (xp|xp) from ovov (EA: x=i occupied, p=b virtual: ovov[i][b][i][b];
// IP: x=a virtual, p=j occupied: ovov[j][a][j][a]); K[x][p] = (xx|pp) from oovv
// (EA: oovv[i][i][b][b]; IP: oovv[j][j][a][a]).
__global__ void k_jk(const double* ovov, const double* oovv, int O, int V, int ea, double* J,
                     double* K) {
    long long total = (long long)O * V;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int i = (int)(e / V), b = (int)(e - (long long)i * V);
        long long ib = (long long)i * V + b;
        double jv = ovov[ib * O * V + ib];
        double kv = oovv[(((long long)i * O + i) * V + b) * V + b];
        if (ea) {
            J[ib] = jv;
            K[ib] = kv;
        } else {
            J[(long long)b * O + i] = jv;
            K[(long long)b * O + i] = kv;
        }
    }
}

void diag22_first_order(adc_ctx* c, double* d) {
    Engine& E = c->E;
    const int O = c->O, V = c->V, Q = c->Q;
    const bool ea = c->kind == ADC_EA;
    const int np = (int)c->n2p;
    const long long nx = c->n2x;
    DBuf<double> J, K, Dpp, Epp;
    J.alloc((size_t)O * V, &c->arena);
    K.alloc((size_t)O * V, &c->arena);
    Dpp.alloc((size_t)np * np, &c->arena);
    Epp.alloc((size_t)np * np, &c->arena);
    hipLaunchKernelGGL(k_jk, dim3(nblk((long long)O * V, 256)), dim3(256), 0, E.stream, c->ovov.p,
                       c->oovv.p, O, V, ea ? 1 : 0, J.p, K.p);
    hipLaunchKernelGGL(k_pair_ints, dim3(nblk((long long)np * np, 256)), dim3(256), 0, E.stream,
                       ea ? c->Bvv.p : c->Boo.p, np, Q, Dpp.p, Epp.p);
    long long total = nx * np * np;
    hipLaunchKernelGGL(k_diag22_first, dim3(nblk(total, 256)), dim3(256), 0, E.stream,
                       d + c->n1, nx, np, ea ? c->eo.p : c->ev.p, ea ? c->ev.p : c->eo.p,
                       ea ? -1.0 : 1.0, ea ? 1.0 : -1.0, J.p, K.p, Dpp.p, Epp.p, ea ? 1 : 0);
    ADC_HIP(hipGetLastError());
    ADC_HIP(hipStreamSynchronize(E.stream));
}

}  // namespace adc
