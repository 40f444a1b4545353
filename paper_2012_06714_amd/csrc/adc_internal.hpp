// Internal declarations of the ADC library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/adc.h"

namespace adc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define ADC_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::adc::Error(e_ == hipErrorOutOfMemory ? ADC_E_OOM : ADC_E_HIP,      \
                               std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

#define ADC_BLAS(call)                                                                 \
    do {                                                                               \
        rocblas_status s_ = (call);                                                    \
        if (s_ != rocblas_status_success)                                              \
            throw ::adc::Error(ADC_E_HIP, std::string(#call " failed: ") +             \
                                              rocblas_status_to_string(s_));           \
    } while (0)

#define ADC_REQUIRE(cond, msg)                                  \
    do {                                                        \
        if (!(cond)) throw ::adc::Error(ADC_E_ARG, (msg));      \
    } while (0)

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
struct Arena;   // tracks the bytes a context owns

template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    Arena* arena = nullptr;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept { swap(o); }
    DBuf& operator=(DBuf&& o) noexcept { swap(o); return *this; }
    ~DBuf() { release(); }
    void swap(DBuf& o) noexcept { std::swap(p, o.p); std::swap(n, o.n); std::swap(arena, o.arena); }
    void alloc(size_t count, Arena* a);
    // at least `count` elements, reallocating only to grow (contents lost then)
    void ensure(size_t count, Arena* a) {
        if (n < count) alloc(count, a);
    }
    void release();
    T* get() const { return p; }
    size_t bytes() const { return n * sizeof(T); }
};

struct Arena {
    size_t used = 0;
    size_t peak = 0;
    size_t limit = SIZE_MAX;
};

template <typename T>
void DBuf<T>::alloc(size_t count, Arena* a) {
    release();
    if (count == 0) return;
    size_t b = count * sizeof(T);
    if (a && a->used + b > a->limit)
        throw Error(ADC_E_OOM, "workspace limit exceeded");
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, b);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(ADC_E_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
    p = static_cast<T*>(q);
    n = count;
    arena = a;
    if (a) {
        a->used += b;
        if (a->used > a->peak) a->peak = a->used;
    }
}

template <typename T>
void DBuf<T>::release() {
    if (p) {
        (void)hipFree(p);
        if (arena) arena->used -= n * sizeof(T);
    }
    p = nullptr;
    n = 0;
}

// Scratch slots reused by the contraction helper (grown on demand).
// While `touched` is set, get() records each slot used with its address and
// size: work recorded with those addresses (a captured graph) stays valid as
// long as every recorded slot still has that address and at least that size.
struct Scratch {
    std::map<int, DBuf<char>> slots;
    Arena* arena = nullptr;
    std::map<int, std::pair<void*, size_t>>* touched = nullptr;
    void* get(int slot, size_t bytes) {
        auto& b = slots[slot];
        if (b.n < bytes) {
            b.release();
            b.alloc(bytes + bytes / 8, arena);
        }
        if (touched) (*touched)[slot] = {b.p, b.n};
        return b.p;
    }
    bool still_valid(const std::map<int, std::pair<void*, size_t>>& rec) const {
        for (const auto& kv : rec) {
            auto it = slots.find(kv.first);
            if (it == slots.end() || it->second.p != kv.second.first ||
                it->second.n < kv.second.second)
                return false;
        }
        return true;
    }
    void erase(int slot) { slots.erase(slot); }
    size_t size_of(int slot) const {
        auto it = slots.find(slot);
        return it == slots.end() ? 0 : it->second.bytes();
    }
    void clear() { slots.clear(); }
};

// ---------------------------------------------------------------------------
// tensor contraction helper: C = beta*C + alpha * sum A*B  (einsum semantics)
// Index letters: i..o occupied (extent O), a..h virtual (extent V), Q auxiliary,
// z vectors, other letters need an explicit extent in Ext.
// ---------------------------------------------------------------------------
struct Ext {
    long long O = 0, V = 0, Q = 0, Z = 0;
    std::map<char, long long> extra;
    long long of(char c) const;
};

struct Engine {
    hipStream_t stream = nullptr;
    rocblas_handle blas = nullptr;
    Scratch scratch;
    Ext ext;
    long long gemm_flops = 0;
    bool bf16 = false;       // FP32 contractions multiply in BF16 (mixed-precision sigma)
    // GEMM tile autotuner: shape key -> fastest tile configuration
    bool autotune = true;
    bool tune_log = false;
    std::map<std::array<long long, 12>, int> tuned;
    hipEvent_t tev[2] = {nullptr, nullptr};
    bool timing = false;     // record events around the particle-particle kernels
    bool ctr_log = false;    // time every contraction and print its GEMM plan to stderr
    int force_cfg = -1;      // GEMM tile configuration forced on every product (-1: automatic)
    long long slice_budget = 1LL << 28;   // elements per operand view of ctr_sliced
    double pp_ms = 0.0;      // accumulated milliseconds of those kernels
};

template <typename T>
void ctr(Engine& E, T alpha, const char* sa, const T* A, const char* sb, const T* B, T beta,
         const char* sc, T* C);

// The same contraction restricted to slices: every letter of `sl` takes the
// values [lo, lo + n) in every operand that carries it (a summed letter sums
// over that range only).  Operands are full tensors with the engine's extents;
// a view that is not contiguous is gathered into scratch, a non-contiguous
// output slice computed in scratch and scattered back.  Views larger than
// `budget` elements (<= 0: the engine's slice_budget) are split further along
// their longest axis, so no temporary exceeds the budget.
struct Slice {
    char c;
    long long lo, n;
};
template <typename T>
void ctr_sliced(Engine& E, T alpha, const char* sa, const T* A, const char* sb, const T* B, T beta,
                const char* sc, T* C, const std::vector<Slice>& sl = {}, long long budget = 0);

// Permute-accumulate: out[so] = beta*out + alpha*in[si]  (same letters).
template <typename T>
void permute(Engine& E, T alpha, const char* si, const T* in, T beta, const char* so, T* out);

// Row-major GEMM on the engine's stream: C[M,N] = alpha op(A) op(B) + beta C, strided batches.
template <typename T>
void gemm_rm(Engine& E, bool ta, bool tb, long long M, long long N, long long K, T alpha,
             const T* A, long long lda, long long sA, const T* B, long long ldb, long long sB,
             T beta, T* C, long long ldc, long long sC, long long batch);

// elementwise helpers (kernels in tensor.hip)
template <typename T> void fill(Engine& E, T* p, T v, size_t n);
template <typename T> void axpy(Engine& E, T a, const T* x, T* y, size_t n);   // y += a x
void convert_d2f(Engine& E, const double* in, float* out, size_t n);
void convert_f2d(Engine& E, const float* in, double* out, size_t n, double beta_out);

}  // namespace adc
