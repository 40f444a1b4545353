// Operands of the EA sigma rearranged for the matrix cores.
//
// The 2p1h-2p1h and coupling terms of EA-ADC(3) (the second-order coupling
// and first-order 2p1h-2p1h rows of Eq. 36) contract the trial vectors with
// t2, t~2 and the (ov|ov), (oo|vv) integrals over an occupied-virtual index
// pair.  Written as products whose summed pair is the contiguous trailing
// run of both operands, every one of them is a single NT product: the
// amplitude and integral sides are permuted once here, the trial-vector side
// once per sigma call (ea_pairs), and the results are scattered straight
// into the sigma layout by the product's output index map.
#include "context.hpp"

#include <algorithm>

namespace adc {

// ---------------------------------------------------------------------------
// per-call pair tensors of the trial vectors
// ---------------------------------------------------------------------------
// One block handles a 32 x 32 tile (x0.., y0..) of the (x, y) plane of Y[z][j]:
// the tile and its mirror (y0.., x0..) go through LDS, and each output row
// [z][x][j][y0..y0+31] is written with consecutive y.
template <typename T, typename TB>
__global__ void k_ea_pairs(const T* __restrict__ Y, int O, int V, int ntx, TB* __restrict__ P1,
                           TB* __restrict__ P2, TB* __restrict__ D, TB* __restrict__ Pm,
                           T* __restrict__ Dw) {
    __shared__ T a[32][33];
    __shared__ T b[32][33];
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    const int x0 = (blockIdx.x / ntx) * 32, y0 = (blockIdx.x % ntx) * 32;
    const int j = blockIdx.y;
    const long long z = blockIdx.z;
    const long long VV = (long long)V * V;
    const T* Yz = Y + (z * O + j) * VV;
    for (int r = ty; r < 32; r += 8) {
        const int x = x0 + r, y = y0 + tx;
        a[r][tx] = (x < V && y < V) ? Yz[(long long)x * V + y] : T(0);   // Y[x][y]
        const int xm = y0 + r, ym = x0 + tx;
        b[r][tx] = (xm < V && ym < V) ? Yz[(long long)xm * V + ym] : T(0);   // Y[y][x]
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int x = x0 + r, y = y0 + tx;
        if (x >= V || y >= V) continue;
        const T p1 = a[r][tx];       // Y[z][j][x][y]
        const T p2 = b[tx][r];       // Y[z][j][y][x]
        const long long o = ((z * V + x) * O + j) * V + y;
        const T d = p2 - T(2) * p1;
        if (P1) P1[o] = (TB)p1;
        if (P2) P2[o] = (TB)p2;
        if (D) D[o] = (TB)d;
        if (Pm) Pm[o] = (TB)(T(2) * p1 - p2);
        if (Dw) Dw[o] = d;
    }
}

template <typename T, typename TB>
void ea_pairs(Engine& E, const T* Y, int nvec, int O, int V, TB* P1, TB* P2, TB* D, TB* Pm, T* Dw) {
    if (nvec <= 0) return;
    const int nt = (V + 31) / 32;
    ADC_REQUIRE(nvec <= 65535 && O <= 65535, "ea_pairs: grid too large");
    dim3 grid((unsigned)(nt * nt), (unsigned)O, (unsigned)nvec);
    hipLaunchKernelGGL((k_ea_pairs<T, TB>), grid, dim3(32, 8), 0, E.stream, Y, O, V, nt, P1, P2, D,
                       Pm, Dw);
    ADC_HIP(hipGetLastError());
}

template void ea_pairs<double, double>(Engine&, const double*, int, int, int, double*, double*,
                                       double*, double*, double*);
template void ea_pairs<float, bf16_t>(Engine&, const float*, int, int, int, bf16_t*, bf16_t*,
                                      bf16_t*, bf16_t*, float*);
template void ea_pairs<float, float>(Engine&, const float*, int, int, int, float*, float*, float*,
                                     float*, float*);

// ---------------------------------------------------------------------------
// resident operands
// ---------------------------------------------------------------------------
// BF16 copy through FP32: the value an FP32 copy would be rounded to when a
// product stages it
__global__ void k_to_bf16(const double* __restrict__ in, bf16_t* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = (bf16_t)(float)in[i];
}
__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

static unsigned grid_of(size_t n) {
    size_t g = (n + 255) / 256;
    return (unsigned)std::min<size_t>(std::max<size_t>(g, 1), 1u << 20);
}

static void to_bf16(adc_ctx* c, const DBuf<double>& src, DBuf<bf16_t>& dst) {
    dst.alloc(src.n, &c->arena);
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_of(src.n)), dim3(256), 0, c->E.stream, src.p, dst.p,
                       src.n);
    ADC_HIP(hipGetLastError());
}
static void to_f32(adc_ctx* c, const DBuf<double>& src, DBuf<float>& dst) {
    dst.alloc(src.n, &c->arena);
    hipLaunchKernelGGL(k_to_f32, dim3(grid_of(src.n)), dim3(256), 0, c->E.stream, src.p, dst.p,
                       src.n);
    ADC_HIP(hipGetLastError());
}

// bytes the arranged operands still to be made would take
static size_t layout_bytes(const adc_ctx* c, int level) {
    const size_t O = c->O, V = c->V, Q = c->Q;
    const size_t big = O * O * V * V, g = O * O * O * V, bvo = c->Bvo.p ? 0 : O * V * Q;
    size_t b = 0;
    if (!c->eal.ready) b += 6 * big * 8 + g * 8 + bvo * 8 + 2 * O * V * Q * 8;
    const size_t f32_small = (c->eal.fG.p ? 0 : g * 4) + (c->fBvo.p ? 0 : O * V * Q * 4) +
                             (c->eal.fH.p ? 0 : 2 * O * V * Q * 4);
    if (level == 1 && !c->eal.ready_mixed) b += 7 * big * 2 + f32_small;
    if (level == 2 && !c->eal.ready_f32) b += 6 * big * 4 + f32_small;
    return b;
}

bool ea_layout_use(adc_ctx* c, int level) {
    c->eal.mode = 0;
    if (c->kind != ADC_EA) return false;
    if (c->ea_layout == 0) {
        if (c->bvv_host)
            throw Error(ADC_E_STATE, "ea_layout 0 reads B_vv on the device: with bvv_host = 1 "
                                     "use ea_layout -1, 1 or 2");
        return false;
    }
    if (c->order == 2 || c->ea_layout == 1 || c->ea_layout == 2) {
        c->eal.mode = c->order == 2 ? 1 : c->ea_layout;
        return true;
    }
    c->eal.mode = 1;
    if (c->eal.ready && (level == 0 || (level == 1 && c->eal.ready_mixed) ||
                         (level == 2 && c->eal.ready_f32)))
        return true;
    if (c->eal.ready_blocked) {   // once blocked, stay blocked (t~ may be released)
        c->eal.mode = 2;
        return true;
    }
    // automatic: the operands still to be made must fit in half the free memory,
    // else their blocks are made per call
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        fr = 0;
    }
    if (layout_bytes(c, level) > fr / 2) c->eal.mode = 2;
    return true;
}

void ea_layout_build(adc_ctx* c, int level) {
    if (c->kind != ADC_EA) return;
    Engine& E = c->E;
    const size_t O = c->O, V = c->V, Q = c->Q;
    const size_t big = O * O * V * V;
    auto& L = c->eal;
    if (c->order != 3) return;    // ADC(2) needs no rearranged operands
    // B_ov as [a][k][Q] for the coupling term that sums over (k, Q)
    if (!c->Bvo.p) {
        c->Bvo.alloc(O * V * Q, &c->arena);
        permute<double>(E, 1.0, "kaQ", c->Bov.p, 0.0, "akQ", c->Bvo.p);
    }
    if (L.mode == 2 && !L.ready && !L.ready_blocked) {
        // blocked path: only the small operands stay resident; t~ and t~ + u~
        // (read per call through t, and once per solve) leave the device
        L.G.alloc(O * O * O * V, &c->arena);
        permute<double>(E, -2.0, "jlka", c->ooov.p, 0.0, "ajkl", L.G.p);
        permute<double>(E, 1.0, "jkla", c->ooov.p, 1.0, "ajkl", L.G.p);
        ensure_tt(c);
        L.H.alloc(O * V * Q, &c->arena);
        ctr_sliced<double>(E, 1.0, "ikbd", c->tt.p, "kdQ", c->Bov.p, 0.0, "ibQ", L.H.p);
        L.BH.alloc(O * V * Q, &c->arena);
        ADC_HIP(hipMemcpyAsync(L.BH.p, c->Bov.p, O * V * Q * sizeof(double),
                               hipMemcpyDeviceToDevice, E.stream));
        axpy<double>(E, 1.0, L.H.p, L.BH.p, O * V * Q);
        ADC_HIP(hipStreamSynchronize(E.stream));
        c->tt.release();
        // only the sliced contraction's own slots: this runs inside a sigma
        // call whose input and result slots are already in use
        for (int slot : {60, 61, 62}) E.scratch.erase(slot);
        if (c->ttu.p && !c->ttu_host) {
            void* h = nullptr;
            ADC_HIP(hipHostMalloc(&h, c->ttu.bytes(), hipHostMallocDefault));
            c->ttu_host = static_cast<double*>(h);
            ADC_HIP(hipMemcpyAsync(h, c->ttu.p, c->ttu.bytes(), hipMemcpyDeviceToHost, E.stream));
            ADC_HIP(hipStreamSynchronize(E.stream));
            c->ttu.release();
        }
        L.ready_blocked = true;
    }
    if (L.mode == 1 && !L.ready) {
        ensure_tt(c);
        L.ttT1.alloc(big, &c->arena);
        permute<double>(E, 1.0, "jkcd", c->tt.p, 0.0, "kdjc", L.ttT1.p);
        L.ttT2.alloc(big, &c->arena);
        permute<double>(E, 1.0, "jkdc", c->tt.p, 0.0, "kdjc", L.ttT2.p);
        L.tT1.alloc(big, &c->arena);
        permute<double>(E, 1.0, "jkcd", c->t.p, 0.0, "kdjc", L.tT1.p);
        L.tD.alloc(big, &c->arena);
        permute<double>(E, 1.0, "ikda", c->t.p, 0.0, "iakd", L.tD.p);
        L.oovvT.alloc(big, &c->arena);
        permute<double>(E, 1.0, "jibc", c->oovv.p, 0.0, "ibjc", L.oovvT.p);
        L.tT.alloc(big, &c->arena);
        permute<double>(E, 1.0, "klab", c->t.p, 0.0, "abkl", L.tT.p);
        L.G.alloc(O * O * O * V, &c->arena);
        permute<double>(E, -2.0, "jlka", c->ooov.p, 0.0, "ajkl", L.G.p);
        permute<double>(E, 1.0, "jkla", c->ooov.p, 1.0, "ajkl", L.G.p);
        // t~ is symmetric under the exchange of its (occupied, virtual) pairs, so
        // H = t~ B_ov serves both sides: sum_kd t~_ik^bd (kd|Q) and sum_kd t~_ki^db (kd|Q)
        L.H.alloc(O * V * Q, &c->arena);
        gemm_map<double, double>(E, false, false, O * V, Q, O * V, 1.0, L.ttT1.p, O * V, c->Bov.p,
                                 Q, 0.0, L.H.p, GemmOut::rowmajor(Q));
        L.BH.alloc(O * V * Q, &c->arena);
        ADC_HIP(hipMemcpyAsync(L.BH.p, c->Bov.p, O * V * Q * sizeof(double),
                               hipMemcpyDeviceToDevice, E.stream));
        axpy<double>(E, 1.0, L.H.p, L.BH.p, O * V * Q);
        L.ready = true;
    }
    if (level >= 1) {
        if (!c->fBvo.p) to_f32(c, c->Bvo, c->fBvo);
        if (!L.fG.p) to_f32(c, L.G, L.fG);
        if (!L.fH.p) to_f32(c, L.H, L.fH);
        if (!L.fBH.p) to_f32(c, L.BH, L.fBH);
    }
    if (L.mode == 1 && level == 2 && !L.ready_f32) {
        to_f32(c, L.ttT1, L.fttT1);
        to_f32(c, L.ttT2, L.fttT2);
        to_f32(c, L.tT1, L.ftT1);
        to_f32(c, L.tD, L.ftD);
        to_f32(c, L.oovvT, L.foovvT);
        to_f32(c, L.tT, L.ftT);
        L.ready_f32 = true;
    }
    if (L.mode == 1 && level == 1) {
        if (!L.ready_mixed) {
            to_bf16(c, L.ttT1, L.httT1);
            to_bf16(c, L.ttT2, L.httT2);
            to_bf16(c, L.tT1, L.htT1);
            to_bf16(c, L.tD, L.htD);
            to_bf16(c, L.oovvT, L.hoovvT);
            to_bf16(c, L.tT, L.htT);
            to_bf16(c, c->ovov, L.hovov);
            L.ready_mixed = true;
        }
    }
}

}  // namespace adc
