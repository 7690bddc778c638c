// CPU stand-in for <hip/hip_runtime.h>, used only by the CPU emulation build
// of the library's kernels (tests/cpuemu).  Every GPU lane runs as a fiber on
// one host thread; wave operations (ballot, readlane, DPP row shifts,
// shuffles, wave barriers) and workgroup barriers are rendezvous points where
// the scheduler waits for every live lane of the wave (or workgroup), so a
// wave operation reached by only part of a wave, or a barrier reached by
// only part of a workgroup, is reported instead of silently mis-executing.
// Device memory is host memory (AddressSanitizer checks every access).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

using std::isfinite;
using std::isnan;

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_uint3 {
    unsigned x, y, z;
};
struct float4 {
    float x, y, z, w;
};
struct longlong2 {
    long long x, y;
};
inline float4 make_float4(float a, float b, float c, float d) { return float4{a, b, c, d}; }

inline int max(int a, int b) { return a > b ? a : b; }
inline int min(int a, int b) { return a < b ? a : b; }

namespace emu {
emu_uint3 &thread_idx();
extern emu_uint3 g_block_idx;
extern dim3 g_block_dim, g_grid_dim;
void *dyn_shared();

// wave operations (all rendezvous over the live lanes of the wave)
enum Op { OP_BALLOT = 1, OP_READLANE, OP_FIRSTLANE, OP_DPP, OP_SHFL_UP, OP_SHFL_XOR, OP_WAVE_BARRIER, OP_SHFL };
uint64_t wave_op(int op, uint64_t v, int64_t a0, int64_t a1, int64_t a2, const void *site);
void block_barrier(const void *site);
int lane();

void launch(dim3 grid, dim3 block, size_t shmem, std::function<void()> body);
} // namespace emu

#define threadIdx (emu::thread_idx())
#define blockIdx (emu::g_block_idx)
#define blockDim (emu::g_block_dim)
#define gridDim (emu::g_grid_dim)

#define EMU_SITE (__builtin_return_address(0))

__attribute__((noinline)) inline uint64_t __ballot(int pred)
{
    return emu::wave_op(emu::OP_BALLOT, pred ? 1u : 0u, 0, 0, 0, EMU_SITE);
}
inline unsigned __lane_id() { return (unsigned)emu::lane(); }
__attribute__((noinline)) inline void __syncthreads() { emu::block_barrier(EMU_SITE); }

__attribute__((noinline)) inline int emu_readlane(int v, int l)
{
    return (int)(uint32_t)emu::wave_op(emu::OP_READLANE, (uint32_t)v, l, 0, 0, EMU_SITE);
}
__attribute__((noinline)) inline int emu_readfirstlane(int v)
{
    return (int)(uint32_t)emu::wave_op(emu::OP_FIRSTLANE, (uint32_t)v, 0, 0, 0, EMU_SITE);
}
// DPP on 32-bit values: a0 = control, a1 = old value, a2 = bound_ctrl
__attribute__((noinline)) inline int emu_update_dpp(int old, int v, int ctrl, int rm, int bm, bool bc)
{
    if (rm != 0xf || bm != 0xf) {
        fprintf(stderr, "cpuemu: DPP row/bank masks other than 0xf are not emulated\n");
        abort();
    }
    return (int)(uint32_t)emu::wave_op(emu::OP_DPP, (uint32_t)v, ctrl, (uint32_t)old, bc ? 1 : 0, EMU_SITE);
}
__attribute__((noinline)) inline void emu_wave_barrier()
{
    emu::wave_op(emu::OP_WAVE_BARRIER, 0, 0, 0, 0, EMU_SITE);
}
#define __builtin_amdgcn_readlane(v, l) emu_readlane((int)(v), (int)(l))
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane((int)(v))
#define __builtin_amdgcn_update_dpp(old, v, ctrl, rm, bm, bc) emu_update_dpp((old), (v), (ctrl), (rm), (bm), (bc))
#define __builtin_amdgcn_mov_dpp(v, ctrl, rm, bm, bc) emu_update_dpp(0, (v), (ctrl), (rm), (bm), (bc))
#define __builtin_amdgcn_wave_barrier() emu_wave_barrier()
#define __builtin_amdgcn_fence(order, scope) ((void)(order), (void)(scope))
inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }

template <class T>
__attribute__((noinline)) T emu_shfl(int op, T v, int a)
{
    static_assert(sizeof(T) == 4, "32-bit shuffles only");
    uint32_t b;
    memcpy(&b, &v, 4);
    uint32_t r = (uint32_t)emu::wave_op(op, b, a, 0, 0, EMU_SITE);
    T out;
    memcpy(&out, &r, 4);
    return out;
}
template <class T>
T __shfl_up(T v, unsigned delta) { return emu_shfl<T>(emu::OP_SHFL_UP, v, (int)delta); }
template <class T>
T __shfl_xor(T v, int mask) { return emu_shfl<T>(emu::OP_SHFL_XOR, v, mask); }
template <class T>
T __shfl(T v, int src) { return emu_shfl<T>(emu::OP_SHFL, v, src); }

// bit casts and bit counts
inline int __float_as_int(float f) { int i; memcpy(&i, &f, 4); return i; }
inline unsigned __float_as_uint(float f) { unsigned i; memcpy(&i, &f, 4); return i; }
inline float __int_as_float(int i) { float f; memcpy(&f, &i, 4); return f; }
inline float __uint_as_float(unsigned i) { float f; memcpy(&f, &i, 4); return f; }
inline long long __double_as_longlong(double d) { long long i; memcpy(&i, &d, 8); return i; }
inline double __longlong_as_double(long long i) { double d; memcpy(&d, &i, 8); return d; }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline int __ffsll(unsigned long long v) { return __builtin_ffsll((long long)v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline int __ffs(int v) { return __builtin_ffs(v); }
inline int __ffs(unsigned v) { return __builtin_ffs((int)v); }
inline int __clz(int v) { return v == 0 ? 32 : __builtin_clz((unsigned)v); }
inline int __clzll(long long v) { return v == 0 ? 64 : __builtin_clzll((unsigned long long)v); }

// atomics: fibers run on one host thread, but the builtins keep them honest
template <class T>
T atomicAdd(T *p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline float atomicAdd(float *p, float v) { float o = *p; *p = o + v; return o; }
inline double atomicAdd(double *p, double v) { double o = *p; *p = o + v; return o; }
template <class T>
T atomicMax(T *p, T v) { T o = *p; if (v > o) *p = v; return o; }
template <class T>
T atomicMin(T *p, T v) { T o = *p; if (v < o) *p = v; return o; }
template <class T>
T atomicOr(T *p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
template <class T>
T atomicExch(T *p, T v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
template <class T>
T atomicCAS(T *p, T cmp, T v) { __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST); return cmp; }
#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_SYSTEM 4
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_max(p, v, order, scope) atomicMax((p), (v))
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_exchange(p, v, order, scope) __atomic_exchange_n((p), (v), __ATOMIC_SEQ_CST)

// ------------------------------------------------------------ host API
typedef int hipError_t;
typedef void *hipStream_t;
typedef void *hipEvent_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1, hipErrorNotSupported = 801 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum { hipHostMallocDefault = 0 };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };

hipError_t hipMalloc(void **p, size_t bytes);
template <class T>
hipError_t hipMalloc(T **p, size_t bytes) { return hipMalloc((void **)p, bytes); }
hipError_t hipFree(void *p);
hipError_t hipMallocAsync(void **p, size_t bytes, hipStream_t);
hipError_t hipFreeAsync(void *p, hipStream_t);
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void *p);
hipError_t hipMemsetAsync(void *p, int v, size_t bytes, hipStream_t s = nullptr);
hipError_t hipMemset(void *p, int v, size_t bytes);
hipError_t hipMemsetD32Async(void *p, int v, size_t count, hipStream_t s = nullptr);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s = nullptr);
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
hipError_t hipPeekAtLastError();
const char *hipGetErrorString(hipError_t);
hipError_t hipGetDevice(int *d);
struct hipDeviceProp_t {
    char gcnArchName[256];
};
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int d);
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 63 };
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int d);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *f, int threads, size_t lds);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
enum { hipEventDefault = 0, hipEventDisableTiming = 2 };
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipFuncSetAttribute(const void *f, hipFuncAttribute a, int v);
hipError_t hipGetSymbolAddress(void **p, const void *sym);
#define HIP_SYMBOL(x) (&(x))
// streams and graphs: stream capture is not emulated (it reports an error,
// so callers take their direct-launch path)
typedef void *hipGraph_t;
typedef void *hipGraphExec_t;
typedef void *hipGraphNode_t;
enum { hipStreamNonBlocking = 1 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *n, char *log, size_t len);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);

#define hipLaunchKernelGGL(K, G, B, S, ST, ...) emu::launch(dim3(G), dim3(B), (size_t)(S), [=]() { K(__VA_ARGS__); })
