// Out-of-core B_vv (the paper's out-of-core storage mode, Sec. III.A, for the
// three-index factors of the largest block): with option "bvv_host" the vv
// block of the DF factors, and its FP32 / BF16 copies for the reduced-precision
// sigma, live in pinned host memory; every product that reads it stages the
// rows it needs into a device buffer, one block of rows at a time (copies on
// the context's stream, ordered with the products that read them).
#include "context.hpp"

#include <algorithm>

namespace adc {

namespace {

template <typename TO>
__global__ void k_narrow_rows(const double* __restrict__ in, TO* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if constexpr (sizeof(TO) == 2)
            out[i] = (TO)(float)in[i];   // BF16 through FP32, as the resident copies
        else
            out[i] = (TO)in[i];
    }
}

template <typename T>
T* host_ptr(adc_ctx* c);
template <>
double* host_ptr<double>(adc_ctx* c) { return c->hB64; }
template <>
float* host_ptr<float>(adc_ctx* c) { return c->hB32; }
template <>
bf16_t* host_ptr<bf16_t>(adc_ctx* c) { return c->hB16; }

template <typename T>
T*& host_slot(adc_ctx* c);
template <>
double*& host_slot<double>(adc_ctx* c) { return c->hB64; }
template <>
float*& host_slot<float>(adc_ctx* c) { return c->hB32; }
template <>
bf16_t*& host_slot<bf16_t>(adc_ctx* c) { return c->hB16; }

size_t bvv_elems(const adc_ctx* c) { return (size_t)c->V * c->V * c->Q; }

// pinned host copy of type T made from the FP64 host copy, a block of rows at
// a time through the device
template <typename T>
void ensure_host(adc_ctx* c) {
    if constexpr (sizeof(T) == 8) return;   // the FP64 copy is the one moved out
    T*& h = host_slot<T>(c);
    if (h) return;
    Engine& E = c->E;
    void* p = nullptr;
    ADC_HIP(hipHostMalloc(&p, bvv_elems(c) * sizeof(T), hipHostMallocDefault));
    h = static_cast<T*>(p);
    const long long rows = (long long)c->V * c->V, Q = c->Q;
    const long long nb = bvv_chunk_rows(c, sizeof(double));
    DBuf<double> in;
    DBuf<T> out;
    in.alloc((size_t)(nb * Q), &c->arena);
    out.alloc((size_t)(nb * Q), &c->arena);
    for (long long r0 = 0; r0 < rows; r0 += nb) {
        const long long n = std::min(nb, rows - r0);
        const size_t cnt = (size_t)(n * Q);
        ADC_HIP(hipMemcpyAsync(in.p, c->hB64 + r0 * Q, cnt * sizeof(double),
                               hipMemcpyHostToDevice, E.stream));
        size_t g = std::min<size_t>((cnt + 255) / 256, 1u << 20);
        hipLaunchKernelGGL(k_narrow_rows<T>, dim3((unsigned)g), dim3(256), 0, E.stream, in.p,
                           out.p, cnt);
        ADC_HIP(hipGetLastError());
        ADC_HIP(hipMemcpyAsync(h + r0 * Q, out.p, cnt * sizeof(T), hipMemcpyDeviceToHost,
                               E.stream));
        ADC_HIP(hipStreamSynchronize(E.stream));
    }
}

}  // namespace

long long bvv_chunk_rows(const adc_ctx* c, size_t elem) {
    const long long bytes = c->E.slice_budget * 8;
    return std::max<long long>(1, std::min<long long>((long long)c->V * c->V,
                                                      bytes / ((long long)c->Q * (long long)elem)));
}

void bvv_set_host(adc_ctx* c, bool on) {
    Engine& E = c->E;
    ADC_REQUIRE(c->kind == ADC_EA, "bvv_host: only EA sigma reads B_vv after the setup");
    if (on == c->bvv_host) return;
    drop_graphs(c);
    const size_t n = bvv_elems(c);
    if (on) {
        void* p = nullptr;
        ADC_HIP(hipHostMalloc(&p, n * sizeof(double), hipHostMallocDefault));
        c->hB64 = static_cast<double*>(p);
        ADC_HIP(hipMemcpyAsync(c->hB64, c->Bvv.p, n * sizeof(double), hipMemcpyDeviceToHost,
                               E.stream));
        ADC_HIP(hipStreamSynchronize(E.stream));
        c->Bvv.release();
        c->fBvv.release();   // made again on the host from hB64 when needed
        c->hBvv.release();
        c->bvv_host = true;
    } else {
        c->Bvv.alloc(n, &c->arena);
        ADC_HIP(hipMemcpyAsync(c->Bvv.p, c->hB64, n * sizeof(double), hipMemcpyHostToDevice,
                               E.stream));
        ADC_HIP(hipStreamSynchronize(E.stream));
        for (void* h : {(void*)c->hB64, (void*)c->hB32, (void*)c->hB16})
            if (h) (void)hipHostFree(h);
        c->hB64 = nullptr;
        c->hB32 = nullptr;
        c->hB16 = nullptr;
        c->bvv_host = false;
        c->mixed_ready = false;   // the device FP32 / BF16 copies are made again
    }
    E.scratch.clear();
}

void bvv_release_host(adc_ctx* c) {
    for (void* h : {(void*)c->hB64, (void*)c->hB32, (void*)c->hB16})
        if (h) (void)hipHostFree(h);
    c->hB64 = nullptr;
    c->hB32 = nullptr;
    c->hB16 = nullptr;
}

template <typename T>
const T* bvv_rows(adc_ctx* c, long long r0, long long n, int slot) {
    ensure_host<T>(c);
    Engine& E = c->E;
    const size_t cnt = (size_t)(n * c->Q);
    T* d = (T*)E.scratch.get(slot, cnt * sizeof(T));
    ADC_HIP(hipMemcpyAsync(d, host_ptr<T>(c) + r0 * c->Q, cnt * sizeof(T), hipMemcpyHostToDevice,
                           E.stream));
    return d;
}

template const double* bvv_rows<double>(adc_ctx*, long long, long long, int);
template const float* bvv_rows<float>(adc_ctx*, long long, long long, int);
template const bf16_t* bvv_rows<bf16_t>(adc_ctx*, long long, long long, int);

}  // namespace adc
