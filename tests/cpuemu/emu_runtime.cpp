// Fiber scheduler and host API of the CPU emulation (see hip/hip_runtime.h).
//
// A launch runs its workgroups one after another.  Each lane of a workgroup
// is a fiber with its own stack (switched by emu_switch below, which saves
// the callee-saved registers and swaps stack pointers: no system call); the scheduler resumes every ready
// lane in lane order until it blocks at a rendezvous or returns.  A wave
// rendezvous completes when every live lane of the wave waits at the same
// wave operation (same kind, same call site); a workgroup barrier completes
// when every live lane of the workgroup waits at a barrier.  Any other
// state with no runnable lane is a divergence or deadlock: the scheduler
// prints where each lane waits and aborts.
#include <sanitizer/common_interface_defs.h>
#include <sys/mman.h>

#include <vector>

#include "hip/hip_runtime.h"

// emu_switch(&save_sp, next_sp): push the callee-saved registers, store the
// stack pointer in save_sp, load next_sp, pop that fiber's registers, return
// into it.  x86-64 System V.
extern "C" void emu_switch(void **save_sp, void *next_sp);
asm(R"(
    .text
    .globl emu_switch
    .type emu_switch, @function
emu_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_switch, .-emu_switch
)");

namespace emu {

emu_uint3 g_block_idx;
dim3 g_block_dim, g_grid_dim;
static std::vector<unsigned char> g_dyn;
void *dyn_shared() { return g_dyn.data(); }

enum State { READY, WAIT_WAVE, WAIT_BLOCK, DONE };
constexpr size_t STACK = 512 * 1024;
constexpr int WAVE = 64;

struct Lane {
    void *sp = nullptr; // saved stack pointer while switched out
    void *stack = nullptr;
    void *fake = nullptr;
    emu_uint3 tid;
    int state = DONE;
    int op = 0;
    const void *site = nullptr;
    uint64_t v = 0, res = 0;
    int64_t a0 = 0, a1 = 0, a2 = 0;
    uint64_t last_v = 0; // the lane's most recent deposited value (read by readlane of a dead lane)
};

static std::vector<Lane> g_lanes;
static int g_cur = -1;
static void *g_sched_sp = nullptr;
static const void *g_sched_bottom = nullptr;
static size_t g_sched_size = 0;
static std::function<void()> *g_body = nullptr;
static std::vector<int> g_order;
static uint64_t g_rng = 0;
static bool g_rng_init = false;

emu_uint3 &thread_idx() { return g_lanes[g_cur].tid; }
int lane() { return g_cur % WAVE; }

static void yield_to_sched(bool dying)
{
    Lane &L = g_lanes[g_cur];
    __sanitizer_start_switch_fiber(dying ? nullptr : &L.fake, g_sched_bottom, g_sched_size);
    emu_switch(&L.sp, g_sched_sp);
    __sanitizer_finish_switch_fiber(L.fake, &g_sched_bottom, &g_sched_size);
}

extern "C" void emu_lane_entry()
{
    __sanitizer_finish_switch_fiber(nullptr, &g_sched_bottom, &g_sched_size);
    (*g_body)();
    g_lanes[g_cur].state = DONE;
    yield_to_sched(true);
    abort(); // a finished lane is never resumed
}

// Initial stack of a fiber: six zero registers for emu_switch to pop, then
// emu_lane_entry as the return address, then a dummy return address slot so
// that the entry sees the stack alignment of an ordinary call.
static void *fresh_stack(void *base)
{
    uintptr_t top = ((uintptr_t)base + STACK) & ~(uintptr_t)15;
    void **sp = (void **)top;
    *--sp = nullptr;                        // dummy return address of emu_lane_entry
    *--sp = (void *)&emu_lane_entry;        // emu_switch returns here
    for (int i = 0; i < 6; ++i)
        *--sp = nullptr;                    // rbp rbx r12 r13 r14 r15
    return sp;
}

uint64_t wave_op(int op, uint64_t v, int64_t a0, int64_t a1, int64_t a2, const void *site)
{
    Lane &L = g_lanes[g_cur];
    L.state = WAIT_WAVE;
    L.op = op;
    L.v = v;
    L.last_v = v;
    L.a0 = a0;
    L.a1 = a1;
    L.a2 = a2;
    L.site = site;
    yield_to_sched(false);
    return g_lanes[g_cur].res;
}

void block_barrier(const void *site)
{
    Lane &L = g_lanes[g_cur];
    L.state = WAIT_BLOCK;
    L.site = site;
    yield_to_sched(false);
}

static void report(const char *why, int b0, int b1)
{
    fprintf(stderr, "cpuemu: %s (block %u,%u; lanes %d..%d)\n", why, g_block_idx.x, g_block_idx.y, b0, b1 - 1);
    for (int i = b0; i < b1; ++i) {
        const Lane &L = g_lanes[i];
        fprintf(stderr, "  lane %4d: state %d op %d site %p\n", i, L.state, L.op, L.site);
    }
    abort();
}

// Completes the wave rendezvous of lanes [w0, w1) if every live lane waits at
// the same wave operation.  Returns true if it completed one.
static bool resolve_wave(int w0, int w1)
{
    int live = 0, waiting = 0, blocked = 0;
    int first = -1;
    for (int i = w0; i < w1; ++i) {
        const Lane &L = g_lanes[i];
        if (L.state == DONE)
            continue;
        ++live;
        if (L.state == WAIT_WAVE) {
            ++waiting;
            if (first < 0)
                first = i;
        } else if (L.state == WAIT_BLOCK) {
            ++blocked;
        }
    }
    if (live == 0 || waiting == 0 || waiting + blocked != live)
        return false;
    if (blocked)
        report("part of a wave waits at a wave operation while the rest waits at a workgroup barrier", w0, w1);
    const Lane &F = g_lanes[first];
    for (int i = w0; i < w1; ++i) {
        const Lane &L = g_lanes[i];
        if (L.state == WAIT_WAVE && (L.op != F.op || L.site != F.site))
            report("divergent wave operation: live lanes of one wave wait at different wave operations", w0, w1);
    }
    uint64_t vals[WAVE], active = 0;
    for (int i = w0; i < w1; ++i) {
        const Lane &L = g_lanes[i];
        vals[i - w0] = L.state == WAIT_WAVE ? L.v : L.last_v;
        if (L.state == WAIT_WAVE)
            active |= 1ull << (i - w0);
    }
    const int nl = w1 - w0;
    uint64_t ballot = 0;
    if (F.op == OP_BALLOT)
        for (int i = 0; i < nl; ++i)
            if (((active >> i) & 1) && vals[i])
                ballot |= 1ull << i;
    for (int i = w0; i < w1; ++i) {
        Lane &L = g_lanes[i];
        if (L.state != WAIT_WAVE)
            continue;
        const int me = i - w0;
        uint64_t r = 0;
        switch (F.op) {
        case OP_BALLOT:
            r = ballot;
            break;
        case OP_READLANE: {
            const int src = (int)L.a0;
            if (src < 0 || src >= WAVE) {
                fprintf(stderr, "cpuemu: readlane of lane %d\n", src);
                abort();
            }
            r = src < nl ? vals[src] : 0;
            break;
        }
        case OP_FIRSTLANE:
            r = vals[__builtin_ctzll(active)];
            break;
        case OP_DPP: {
            const int ctrl = (int)L.a0;
            int src = -1;
            if (ctrl >= 0x111 && ctrl <= 0x11f) { // row_shr:1..15
                const int sh = ctrl - 0x110;
                if ((me & 15) >= sh)
                    src = me - sh;
            } else {
                fprintf(stderr, "cpuemu: DPP control 0x%x is not emulated\n", ctrl);
                abort();
            }
            if (src >= 0 && ((active >> src) & 1))
                r = (uint32_t)vals[src];
            else
                r = L.a2 ? 0u : (uint32_t)L.a1;
            break;
        }
        case OP_SHFL_UP: {
            const int src = me - (int)L.a0;
            r = (src >= 0 && ((active >> src) & 1)) ? vals[src] : vals[me];
            break;
        }
        case OP_SHFL_XOR: {
            const int src = me ^ (int)L.a0;
            r = (src < nl && ((active >> src) & 1)) ? vals[src] : vals[me];
            break;
        }
        case OP_SHFL: { // lane-indexed read (ds_bpermute); the source must be active
            const int src = (int)L.a0 & 63;
            if (src >= nl || !((active >> src) & 1)) {
                fprintf(stderr, "cpuemu: __shfl from inactive lane %d\n", src);
                abort();
            }
            r = vals[src];
            break;
        }
        case OP_WAVE_BARRIER:
            break;
        default:
            fprintf(stderr, "cpuemu: unknown wave op %d\n", F.op);
            abort();
        }
        L.res = r;
        L.state = READY;
    }
    return true;
}

void launch(dim3 grid, dim3 block, size_t shmem, std::function<void()> body)
{
    const int nt = (int)(block.x * block.y * block.z);
    if (nt < 1 || nt > 1024 || block.y != 1 || block.z != 1) {
        fprintf(stderr, "cpuemu: unsupported block shape %u x %u x %u\n", block.x, block.y, block.z);
        abort();
    }
    if (grid.z != 1) {
        fprintf(stderr, "cpuemu: 3D grids are not emulated\n");
        abort();
    }
    g_block_dim = block;
    g_grid_dim = grid;
    g_body = &body;
    if ((int)g_lanes.size() < nt) {
        size_t old = g_lanes.size();
        g_lanes.resize(nt);
        for (size_t i = old; i < g_lanes.size(); ++i) {
            g_lanes[i].stack = mmap(nullptr, STACK, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE,
                                    -1, 0);
            if (g_lanes[i].stack == MAP_FAILED) {
                fprintf(stderr, "cpuemu: mmap of a fiber stack failed\n");
                abort();
            }
        }
    }
    g_dyn.assign(shmem ? shmem : 1, 0xA5); // LDS starts as garbage, as on the GPU
    if (g_order.size() != (size_t)nt) {
        g_order.resize(nt);
        for (int i = 0; i < nt; ++i)
            g_order[i] = i;
    }
    if (!g_rng_init) {
        const char *e = getenv("EMU_SEED");
        g_rng = e ? strtoull(e, nullptr, 10) : 12345u;
        g_rng_init = true;
    }
    for (unsigned by = 0; by < grid.y; ++by) {
        for (unsigned bx = 0; bx < grid.x; ++bx) {
            g_block_idx = emu_uint3{bx, by, 0};
            for (int i = 0; i < nt; ++i) {
                Lane &L = g_lanes[i];
                L.tid = emu_uint3{(unsigned)i, 0, 0};
                L.state = READY;
                L.res = L.v = L.last_v = 0;
                L.fake = nullptr;
                L.sp = fresh_stack(L.stack);
            }
            while (true) {
                bool progressed = false;
                // ready lanes resume in a seeded random order: between two
                // rendezvous no lane may rely on another lane having run
                for (int q = nt - 1; q > 0; --q) {
                    g_rng = g_rng * 6364136223846793005ull + 1442695040888963407ull;
                    std::swap(g_order[q], g_order[(int)((g_rng >> 33) % (uint64_t)(q + 1))]);
                }
                for (int qi = 0; qi < nt; ++qi) {
                    const int i = g_order[qi];
                    if (g_lanes[i].state != READY)
                        continue;
                    g_cur = i;
                    void *fake = nullptr;
                    __sanitizer_start_switch_fiber(&fake, g_lanes[i].stack, STACK);
                    emu_switch(&g_sched_sp, g_lanes[i].sp);
                    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
                    progressed = true;
                }
                int live = 0, at_barrier = 0;
                for (int i = 0; i < nt; ++i) {
                    if (g_lanes[i].state != DONE)
                        ++live;
                    if (g_lanes[i].state == WAIT_BLOCK)
                        ++at_barrier;
                }
                if (live == 0)
                    break;
                for (int w0 = 0; w0 < nt; w0 += WAVE)
                    progressed |= resolve_wave(w0, std::min(nt, w0 + WAVE));
                if (at_barrier == live) {
                    for (int i = 0; i < nt; ++i)
                        if (g_lanes[i].state == WAIT_BLOCK)
                            g_lanes[i].state = READY;
                    progressed = true;
                }
                if (!progressed)
                    report("no lane can make progress (a barrier or wave operation not reached by every live lane)",
                           0, nt);
            }
        }
    }
    g_cur = -1;
    g_body = nullptr;
}

} // namespace emu

// ------------------------------------------------------------ host API
static hipError_t g_last = hipSuccess;

hipError_t hipMalloc(void **p, size_t bytes)
{
    *p = malloc(bytes ? bytes : 1);
    if (!*p)
        return hipErrorOutOfMemory;
    memset(*p, 0xCD, bytes); // device memory starts as garbage
    return hipSuccess;
}
hipError_t hipFree(void *p)
{
    free(p);
    return hipSuccess;
}
hipError_t hipMallocAsync(void **p, size_t bytes, hipStream_t) { return hipMalloc(p, bytes); }
hipError_t hipFreeAsync(void *p, hipStream_t) { return hipFree(p); }
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
hipError_t hipHostFree(void *p) { return hipFree(p); }
hipError_t hipMemsetAsync(void *p, int v, size_t bytes, hipStream_t)
{
    memset(p, v, bytes);
    return hipSuccess;
}
hipError_t hipMemset(void *p, int v, size_t bytes) { return hipMemsetAsync(p, v, bytes, nullptr); }
hipError_t hipMemsetD32Async(void *p, int v, size_t count, hipStream_t)
{
    int32_t *q = (int32_t *)p;
    for (size_t i = 0; i < count; ++i)
        q[i] = v;
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t)
{
    memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind k)
{
    return hipMemcpyAsync(dst, src, bytes, k, nullptr);
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError()
{
    hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}
hipError_t hipPeekAtLastError() { return g_last; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int)
{
    strcpy(p->gcnArchName, "cpu-emulation");
    return hipSuccess;
}

// A small emulated device: few persistent workgroups, so that each one
// takes many groups from the work counter.
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int)
{
    *v = 4;
    return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *, int, size_t)
{
    *n = 2;
    return hipSuccess;
}

hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = malloc(8);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    free(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t)
{
    *ms = 0.0f;
    return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipGetSymbolAddress(void **p, const void *sym)
{
    *p = const_cast<void *>(sym);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    *s = malloc(8);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    free(s);
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g)
{
    *g = nullptr;
    return hipErrorNotSupported;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t, hipGraphNode_t *, char *, size_t)
{
    *e = nullptr;
    return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
