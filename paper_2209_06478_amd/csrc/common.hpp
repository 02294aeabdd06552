// Shared internals of libdsm: error plumbing, value-type helpers and
// wavefront/workgroup reduction primitives for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/dsm.h"

#define DSM_API extern "C" __attribute__((visibility("default")))

namespace dsm {

using i32 = int32_t;
using i64 = int64_t;
using u32 = uint32_t;
using u64 = uint64_t;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
const char *last_error_cstr();
void clear_error();

// A failed library step: status + message, thrown only inside the library
// and turned into a dsm_status at the ABI.
struct Error {
    dsm_status status;
    std::string msg;
};

[[noreturn]] void fail(dsm_status s, const std::string &msg);

#define DSM_HIP(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::dsm::fail(e_ == hipErrorOutOfMemory ? DSM_E_NOMEM : DSM_E_DEVICE,          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

#define DSM_CHECK(cond, status, msg)                                                     \
    do {                                                                                 \
        if (!(cond)) ::dsm::fail((status), (msg));                                       \
    } while (0)

// Runs `body` and maps escaping errors to a status (ABI guard).
template <class F>
dsm_status guard(F &&body) {
    clear_error();
    try {
        body();
        return DSM_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return DSM_E_NOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return DSM_E_DEVICE;
    }
}

// ---------------------------------------------------------------- value types
// BF16 is carried as its 16-bit pattern; widening to FP32 is exact.
struct bf16 {
    uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(bf16 v) {
    u32 u = (u32)v.bits << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// Round-to-nearest-even of an FP32 value to BF16 (NaN kept quiet).
__host__ __device__ inline bf16 float_to_bf16(float f) {
    u32 u;
    memcpy(&u, &f, 4);
    bf16 r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        r.bits = (uint16_t)((u >> 16) | 0x40u);
        return r;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    r.bits = (uint16_t)(u >> 16);
    return r;
}

template <class Acc, class V>
__device__ __forceinline__ Acc widen(V v) {
    return (Acc)v;
}
template <>
__device__ __forceinline__ float widen<float, bf16>(bf16 v) {
    return bf16_to_float(v);
}
template <>
__device__ __forceinline__ double widen<double, bf16>(bf16 v) {
    return (double)bf16_to_float(v);
}

// Load of a matrix value or index that is read once per sweep; NT asks for
// a non-temporal (streaming) access so it does not evict reused vectors.
template <class V, bool NT>
__device__ __forceinline__ V ld_stream(const V *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <>
__device__ __forceinline__ bf16 ld_stream<bf16, true>(const bf16 *p) {
    bf16 r;
    r.bits = __builtin_nontemporal_load(&p->bits);
    return r;
}

// Store of a value that no kernel before the next pass over it reads again.
template <class V, bool NT>
__device__ __forceinline__ void st_stream(V *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

inline size_t dtype_size(int dt) { return dt == DSM_F64 ? 8 : dt == DSM_F32 ? 4 : 2; }
inline const char *format_name(int f) {
    static const char *n[] = {"COO", "CSR", "DIA", "ELL", "HYB", "HDC"};
    return (f >= 0 && f < 6) ? n[f] : "?";
}

// ---------------------------------------------------------------- launch shapes
constexpr int WAVE = 64;   // CDNA wavefront width
constexpr int NXCD = 8;    // accelerator complex dies on MI355X

inline unsigned grid_for(i64 n, int per_block) {
    i64 g = (n + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

// Workgroups are dealt to the XCDs round-robin (workgroup b runs on XCD
// b % 8).  Remapping b so that each XCD receives one contiguous range of
// logical tiles keeps neighbouring tiles - and the vector entries they share
// - in the same L2.  Bijective for any nblocks.
__device__ __forceinline__ u32 xcd_tile(u32 b, u32 nblocks) {
    u32 q = nblocks / NXCD, r = nblocks % NXCD;
    u32 x = b % NXCD, local = b / NXCD;
    u32 base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return base + local;
}

// ---------------------------------------------------------------- operand words
// Sixteen zero bytes in device memory (one copy per translation unit): the
// operand address of a product that must vanish (a slot past the last
// diagonal, a column outside the matrix, an entry past the end of a row).
// Loading from here instead of selecting the loaded value keeps every load
// unconditional: the compiler turns a select whose operand is a load into a
// branch around that load, which leaves one load in flight at a time.
static __device__ __align__(16) unsigned char g_zero16[16];

template <class T>
__device__ __forceinline__ const T *zero_ptr() {
    static_assert(sizeof(T) <= 16, "zero word too small");
    return reinterpret_cast<const T *>(g_zero16);
}

// Sixteen 0xff bytes: int32 column sentinels (-1) for index slots past
// the end.
static __device__ __align__(16) unsigned char g_sentinel16[16] = {
    0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff, 0xff};

template <class T>
__device__ __forceinline__ const T *sentinel_ptr() {
    static_assert(sizeof(T) <= 16, "sentinel word too small");
    return reinterpret_cast<const T *>(g_sentinel16);
}

// ---------------------------------------------------------------- reductions
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Sum over groups of W consecutive lanes (W a power of two <= 64); every
// lane of the group receives the group total.
template <int W, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
}

// Workgroup sum with a fixed combination order (deterministic); result valid
// in every thread.  `lds` needs blockDim.x / WAVE slots.
template <class T>
__device__ __forceinline__ T block_sum(T v, T *lds) {
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < nw; i++) s += lds[i];
    return s;
}

}  // namespace dsm
