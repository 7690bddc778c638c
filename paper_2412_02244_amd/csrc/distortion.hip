// Distortion loss of Eq. (1) for fixed centroids and its gradient, for a
// batch of B independent clouds.
//
//   L_b = sum_i D(x_i, c_a(i)),  a(i) = lowest-index nearest centroid
//   dL/dx_i = 2 (x_i - c_a(i)),  dL/dc_j = 2 sum_{i in S_j} (c_j - x_i)
// The assignment is piecewise constant, so it carries no gradient.
//
// Forward: one thread per point scans its cloud's centroids from LDS in FP32
// (FP32 centroids are used as given, so the only error is the distance
// evaluation) and re-decides near ties with canonical FP64 distances; the
// loss is an FP64 sum in a fixed order.  Backward: grad_x is elementwise in
// FP64; grad_c uses exact fixed-point cluster sums (integer atomics), so
// RN(cnt_j c_j - sum x_i) is computed once from the exact value.
#include <mutex>

#include "ekm_internal.hpp"

namespace ekm {

constexpr int DT_THREADS = 256;
constexpr int DT_TILE = 1024;

template <class T, int D>
__global__ void __launch_bounds__(DT_THREADS) k_dist_assign(const T *x, const T *c, int64_t n, int64_t k, int32_t *a)
{
    __shared__ float4 tile[DT_TILE];
    const int64_t b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < n;
    const T *xb = x + b * n * D, *cb = c + b * k * D;
    double xd[D];
    float xf[D];
    for (int i = 0; i < D; ++i) {
        xd[i] = valid ? (double)xb[p * D + i] : 0.0;
        xf[i] = (float)xd[i];
    }
    int best = 0;
    if (sizeof(T) == 4) {
        float s1 = INFINITY, s2 = INFINITY;
        int id1 = 0;
        for (int64_t t0 = 0; t0 < k; t0 += DT_TILE) {
            int tn = (int)((k - t0) < DT_TILE ? (k - t0) : DT_TILE);
            __syncthreads();
            for (int t = threadIdx.x; t < tn; t += blockDim.x) {
                float q[3] = {0.0f, 0.0f, 0.0f};
                for (int i = 0; i < D; ++i)
                    q[i] = (float)cb[(t0 + t) * D + i];
                tile[t] = make_float4(q[0], q[1], q[2], 0.0f);
            }
            __syncthreads();
            for (int t = 0; t < tn; ++t) {
                float4 c4 = tile[t];
                float cc[3] = {c4.x, c4.y, c4.z};
                float sv = sqdist32<D>(xf, cc);
                if (sv < s1) {
                    s2 = s1;
                    s1 = sv;
                    id1 = (int)(t0 + t);
                } else {
                    s2 = fminf(s2, sv);
                }
            }
        }
        best = id1;
        if (valid && !margin_safe(s1, s2, 0.0f)) {
            double bd = INFINITY;
            for (int64_t j = 0; j < k; ++j) {
                double cd[D];
                for (int i = 0; i < D; ++i)
                    cd[i] = (double)cb[j * D + i];
                double Dv = sqdist64<D>(xd, cd);
                if (Dv < bd) {
                    bd = Dv;
                    best = (int)j;
                }
            }
        }
    } else {
        double bd = INFINITY;
        for (int64_t j = 0; j < k; ++j) {
            double cd[D];
            for (int i = 0; i < D; ++i)
                cd[i] = (double)cb[j * D + i];
            double Dv = sqdist64<D>(xd, cd);
            if (Dv < bd) {
                bd = Dv;
                best = (int)j;
            }
        }
    }
    if (valid)
        a[b * n + p] = best;
}

// One block per cloud, fixed summation order.
template <class T, int D>
__global__ void __launch_bounds__(DT_THREADS) k_dist_loss(const T *x, const T *c, const int32_t *a, int64_t n,
                                                          int64_t k, double *loss)
{
    __shared__ double red[DT_THREADS];
    const int64_t b = blockIdx.x;
    const T *xb = x + b * n * D, *cb = c + b * k * D;
    double s = 0.0;
    for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
        int j = a[b * n + p];
        double xd[D], cd[D];
        for (int i = 0; i < D; ++i) {
            xd[i] = (double)xb[p * D + i];
            cd[i] = (double)cb[(int64_t)j * D + i];
        }
        s += sqdist64<D>(xd, cd);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = DT_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss[b] = red[0];
}

template <class T, int D>
__global__ void __launch_bounds__(DT_THREADS) k_dist_gx(const T *x, const T *c, const int32_t *a, const double *g,
                                                        int64_t B, int64_t n, int64_t k, T *gx)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= B * n)
        return;
    int64_t b = q / n;
    int j = a[q];
    double two_g = 2.0 * g[b];
    for (int i = 0; i < D; ++i) {
        double t = (double)x[q * D + i] - (double)c[(b * k + j) * D + i];
        gx[q * D + i] = (T)(two_g * t);
    }
}

// Exact-sum window of the gradient's cluster sums: every coordinate of x and
// c is an integer multiple of 2^-S, S = the largest -(exponent of a lowest set
// bit); the sums need emsb + 1 + S + log2(n) bits.  Computed on the device, so
// the backward pass never waits for the host.
struct WinOut {
    int32_t neg_elsb, emsb, any, status; // status: 0 = ok, 1 = the window is too wide
};

// Clears the accumulators and the window (a fill kernel, not a memset, so
// that the call can be captured into a graph).
__global__ void __launch_bounds__(DT_THREADS) k_dist_zero(int64_t *acc, int64_t nacc, int32_t *cnt, int64_t ncnt,
                                                          WinOut *win)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nacc; q += stride)
        acc[q] = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < ncnt; q += stride)
        cnt[q] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *win = WinOut{-100000, -100000, 0, 0};
}

template <class T>
__device__ inline void window_add(T t, int &ne, int &em, int &any)
{
    if (t != (T)0) {
        int el, eh;
        if (sizeof(T) == 4)
            bits_f32((float)t, el, eh);
        else
            bits_f64((double)t, el, eh);
        ne = max(ne, -el);
        em = max(em, eh);
        any = 1;
    }
}

// Four independent loads per thread and round; one lane per workgroup takes
// part in the atomics.
template <class T>
__global__ void __launch_bounds__(DT_THREADS) k_dist_window(const T *v, int64_t m, const T *w, int64_t mw,
                                                            WinOut *out)
{
    int ne = -100000, em = -100000, any = 0;
    const int64_t tot = m + mw, stride = (int64_t)gridDim.x * blockDim.x;
    auto at = [&](int64_t q) { return q < m ? v[q] : w[q - m]; };
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; q + 3 * stride < tot; q += 4 * stride) {
        const T t0 = at(q), t1 = at(q + stride), t2 = at(q + 2 * stride), t3 = at(q + 3 * stride);
        window_add(t0, ne, em, any);
        window_add(t1, ne, em, any);
        window_add(t2, ne, em, any);
        window_add(t3, ne, em, any);
    }
    for (; q < tot; q += stride)
        window_add(at(q), ne, em, any);
    for (int o = 1; o < WAVE; o <<= 1) {
        ne = max(ne, __shfl_xor(ne, o));
        em = max(em, __shfl_xor(em, o));
        any |= __shfl_xor(any, o);
    }
    __shared__ int red[3][DT_THREADS / WAVE];
    const int wv = (int)threadIdx.x / WAVE;
    if (lane_id() == 0) {
        red[0][wv] = ne;
        red[1][wv] = em;
        red[2][wv] = any;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int u = 1; u < DT_THREADS / WAVE; ++u) {
            ne = max(ne, red[0][u]);
            em = max(em, red[1][u]);
            any |= red[2][u];
        }
        if (any) {
            atomicMax(&out->neg_elsb, ne);
            atomicMax(&out->emsb, em);
            atomicOr(&out->any, 1);
        }
    }
}

// Window checks, identical in every thread that reads the window: the sums
// need emsb + 1 + S + log2(n) bits, and the product cnt * c_j 31 more.
__device__ inline bool window_ok(const WinOut &w, int logn, int &S)
{
    S = w.any ? w.neg_elsb : 0;
    return !w.any || (w.emsb + 1 + S + logn <= MAX_FIX_BITS && w.emsb + 1 + S + 31 <= 125);
}

template <class T, int D>
__global__ void __launch_bounds__(DT_THREADS) k_dist_acc(const T *x, const int32_t *a, int64_t n, int64_t k,
                                                         const WinOut *win, int logn, int64_t *acc, int32_t *cnt)
{
    int S;
    if (!window_ok(*win, logn, S))
        return; // k_dist_gc reports it
    const int64_t b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < n;
    int j = valid ? a[b * n + p] : 0;
    int64_t hi[D], lo[D];
    for (int i = 0; i < D; ++i) {
        T v = valid ? x[(b * n + p) * D + i] : (T)0;
        if (sizeof(T) == 4)
            fix_split_f32((float)v, S, hi[i], lo[i]);
        else
            fix_split_f64((double)v, S, hi[i], lo[i]);
    }
    // points in caller order fall into many clusters per wave: at most two
    // wave reductions, then per-lane atomics
    wave_accumulate_few<D>(valid, j, hi, lo, acc + b * k * D * 2, cnt + b * k, 2);
}

// The same sums with the clusters of one cloud in LDS: workgroup (x, b)
// adds points [x P, (x + 1) P) of cloud b with LDS atomics, then adds its
// non-zero partial sums to the global ones (integer sums: exact in any
// order).  LDS: k (2 D) int64 and k int32.
constexpr int DT_LDS_THREADS = 1024;
constexpr int64_t DT_LDS_POINTS = 16384; // points per workgroup
template <class T, int D>
__global__ void __launch_bounds__(DT_LDS_THREADS) k_dist_acc_lds(const T *x, const int32_t *a, int64_t n, int64_t k,
                                                                 const WinOut *win, int logn, int64_t *acc,
                                                                 int32_t *cnt)
{
    int S;
    if (!window_ok(*win, logn, S))
        return; // k_dist_gc reports it (the whole workgroup returns)
    extern __shared__ int64_t sacc[]; // [k][D][2], then [k] int32 counts
    int32_t *scnt = (int32_t *)(sacc + k * D * 2);
    const int64_t b = blockIdx.y;
    for (int64_t q = threadIdx.x; q < k * D * 2; q += blockDim.x)
        sacc[q] = 0;
    for (int64_t q = threadIdx.x; q < k; q += blockDim.x)
        scnt[q] = 0;
    __syncthreads();
    const int64_t p0 = (int64_t)blockIdx.x * DT_LDS_POINTS;
    const int64_t p1 = p0 + DT_LDS_POINTS < n ? p0 + DT_LDS_POINTS : n;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int j = a[b * n + p];
        for (int i = 0; i < D; ++i) {
            int64_t hi, lo;
            const T v = x[(b * n + p) * D + i];
            if (sizeof(T) == 4)
                fix_split_f32((float)v, S, hi, lo);
            else
                fix_split_f64((double)v, S, hi, lo);
            atomicAdd((unsigned long long *)&sacc[((int64_t)j * D + i) * 2], (unsigned long long)hi);
            atomicAdd((unsigned long long *)&sacc[((int64_t)j * D + i) * 2 + 1], (unsigned long long)lo);
        }
        atomicAdd(&scnt[j], 1);
    }
    __syncthreads();
    int64_t *ab = acc + b * k * D * 2;
    int32_t *cb = cnt + b * k;
    for (int64_t q = threadIdx.x; q < k * D * 2; q += blockDim.x)
        if (sacc[q])
            atomicAdd((unsigned long long *)&ab[q], (unsigned long long)sacc[q]);
    for (int64_t q = threadIdx.x; q < k; q += blockDim.x)
        if (scnt[q])
            atomicAdd(&cb[q], scnt[q]);
}
static size_t dist_acc_lds_bytes(int64_t k, int d) { return (size_t)k * d * 2 * 8 + (size_t)k * 4; }
constexpr size_t DT_LDS_MAX = 64 * 1024; // clusters of a cloud kept in LDS up to this size

template <class T, int D>
__global__ void __launch_bounds__(DT_THREADS) k_dist_gc(const T *c, const double *g, int64_t B, int64_t k,
                                                        WinOut *win, int logn, const int64_t *acc,
                                                        const int32_t *cnt, T *gc)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= B * k)
        return;
    int S;
    const bool ok = window_ok(*win, logn, S);
    if (!ok && q == 0)
        win->status = 1;
    int64_t b = q / k;
    double two_g = 2.0 * g[b];
    int32_t m = cnt[q];
    for (int i = 0; i < D; ++i) {
        if (!ok) { // no exact sum is possible: the gradient is marked invalid
            gc[q * D + i] = (T)NAN;
            continue;
        }
        int64_t ch, cl;
        T cv = c[q * D + i];
        if (sizeof(T) == 4)
            fix_split_f32((float)cv, S, ch, cl);
        else
            fix_split_f64((double)cv, S, ch, cl);
        __int128 Vc = ((__int128)ch << 32) + (__int128)cl;
        __int128 Vs = ((__int128)acc[(q * D + i) * 2] << 32) + (__int128)acc[(q * D + i) * 2 + 1];
        double diff = fix128_to_double(Vc * (__int128)m - Vs, S); // RN(cnt c_j - sum x_i)
        gc[q * D + i] = (T)(two_g * diff);
    }
}

static bool dist_args_ok(const void *x, const void *c, int32_t dtype, int64_t B, int64_t n, int64_t k, int32_t d)
{
    if (!x || !c) {
        set_error("distortion: null pointer");
        return false;
    }
    if (dtype != KM_F32 && dtype != KM_F64) {
        set_error("distortion: dtype must be KM_F32 or KM_F64");
        return false;
    }
    if (B < 1 || n < 1 || k < 1 || (d != 2 && d != 3)) {
        set_error("distortion: need B, n, k >= 1 and d in {2, 3}");
        return false;
    }
    if (B > 65535 || n >= ((int64_t)1 << 31) || k >= ((int64_t)1 << 31)) {
        set_error("distortion: B <= 65535 and n, k < 2^31 required");
        return false;
    }
    return true;
}

template <class T, int D>
static km_status fwd_t(const T *x, const T *c, int64_t B, int64_t n, int64_t k, int32_t *a, double *loss,
                       hipStream_t st)
{
    dim3 grid((unsigned)((n + DT_THREADS - 1) / DT_THREADS), (unsigned)B);
    hipLaunchKernelGGL((k_dist_assign<T, D>), grid, dim3(DT_THREADS), 0, st, x, c, n, k, a);
    hipLaunchKernelGGL((k_dist_loss<T, D>), dim3((unsigned)B), dim3(DT_THREADS), 0, st, x, c, a, n, k, loss);
    return hip_ok(hipGetLastError(), "distortion_fwd launch") ? KM_OK : KM_ERR_HIP;
}

// Scratch of the centroid-gradient sums: [B][k][D][2] int64, [B][k] int32,
// one window record.
size_t dist_scratch_bytes(int64_t B, int64_t k, int d)
{
    return ((size_t)B * k * d * 2 * sizeof(int64_t) + (size_t)B * k * sizeof(int32_t) + 255) / 256 * 256 +
           256;
}

template <class T, int D>
static km_status bwd_t(const T *x, const T *c, const int32_t *a, const double *g, int64_t B, int64_t n, int64_t k,
                       T *gx, T *gc, void *scratch, hipStream_t st)
{
    if (gx) {
        int64_t tot = B * n;
        hipLaunchKernelGGL((k_dist_gx<T, D>), dim3((unsigned)((tot + DT_THREADS - 1) / DT_THREADS)), dim3(DT_THREADS),
                           0, st, x, c, a, g, B, n, k, gx);
        if (!hip_ok(hipGetLastError(), "distortion_bwd launch"))
            return KM_ERR_HIP;
    }
    if (!gc)
        return KM_OK;
    const size_t acc_bytes = (size_t)B * k * D * 2 * sizeof(int64_t);
    const size_t cnt_bytes = (size_t)B * k * sizeof(int32_t);
    char *buf = (char *)scratch;
    int64_t *acc = (int64_t *)buf;
    int32_t *cnt = (int32_t *)(buf + acc_bytes);
    WinOut *win = (WinOut *)(buf + (acc_bytes + cnt_bytes + 255) / 256 * 256);
    int logn = 0;
    while (((int64_t)1 << logn) < n)
        ++logn;
    const int64_t nacc = B * k * D * 2, ncnt = B * k;
    unsigned zb = (unsigned)((nacc + DT_THREADS - 1) / DT_THREADS);
    zb = zb < 1 ? 1 : (zb > 4096 ? 4096 : zb);
    hipLaunchKernelGGL(k_dist_zero, dim3(zb), dim3(DT_THREADS), 0, st, acc, nacc, cnt, ncnt, win);
    const int64_t nwin = B * n * D + B * k * D;
    int64_t wb = (nwin + 4 * DT_THREADS - 1) / (4 * DT_THREADS);
    wb = wb < 1 ? 1 : (wb > 1024 ? 1024 : wb); // few workgroups: their atomics meet on three words
    hipLaunchKernelGGL(k_dist_window<T>, dim3((unsigned)wb), dim3(DT_THREADS), 0, st, x, B * n * D, c, B * k * D,
                       win);
    const size_t lds = dist_acc_lds_bytes(k, D);
    if (lds <= DT_LDS_MAX) {
        dim3 grid((unsigned)((n + DT_LDS_POINTS - 1) / DT_LDS_POINTS), (unsigned)B);
        hipLaunchKernelGGL((k_dist_acc_lds<T, D>), grid, dim3(DT_LDS_THREADS), lds, st, x, a, n, k,
                           (const WinOut *)win, logn, acc, cnt);
    } else {
        dim3 grid((unsigned)((n + DT_THREADS - 1) / DT_THREADS), (unsigned)B);
        hipLaunchKernelGGL((k_dist_acc<T, D>), grid, dim3(DT_THREADS), 0, st, x, a, n, k, (const WinOut *)win, logn,
                           acc, cnt);
    }
    const int64_t tot = B * k;
    hipLaunchKernelGGL((k_dist_gc<T, D>), dim3((unsigned)((tot + DT_THREADS - 1) / DT_THREADS)), dim3(DT_THREADS), 0,
                       st, c, g, B, k, win, logn, (const int64_t *)acc, (const int32_t *)cnt, gc);
    return hip_ok(hipGetLastError(), "distortion_bwd launch") ? KM_OK : KM_ERR_HIP;
}

template <class T, int D>
static km_status bwd_alloc(const T *x, const T *c, const int32_t *a, const double *g, int64_t B, int64_t n,
                           int64_t k, T *gx, T *gc, hipStream_t st)
{
    if (!gc)
        return bwd_t<T, D>(x, c, a, g, B, n, k, gx, gc, nullptr, st);
    // stream-ordered scratch: no host synchronisation
    void *buf = nullptr;
    if (!hip_ok(hipMallocAsync(&buf, dist_scratch_bytes(B, k, D), st), "distortion_bwd: hipMallocAsync"))
        return KM_ERR_OOM;
    km_status s = bwd_t<T, D>(x, c, a, g, B, n, k, gx, gc, buf, st);
    if (!hip_ok(hipFreeAsync(buf, st), "distortion_bwd: hipFreeAsync") && s == KM_OK)
        s = KM_ERR_HIP;
    return s;
}

// Fixed device scratch of distortion_bwd_noalloc: one copy per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host the name is only a stand-in); it uses the device
// address hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and cached.
static km_status noalloc_scratch(void **out)
{
    int dev = 0;
    if (!hip_ok(hipGetDevice(&dev), "distortion_bwd_noalloc: hipGetDevice"))
        return KM_ERR_HIP;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("distortion_bwd_noalloc: device index out of range");
        return KM_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "distortion_bwd_noalloc: hipGetSymbolAddress"))
            return KM_ERR_HIP;
        if (!p) {
            set_error("distortion_bwd_noalloc: hipGetSymbolAddress returned a null address");
            return KM_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KM_OK;
}

} // namespace ekm

using namespace ekm;

extern "C" {

km_status distortion_fwd(const void *x, const void *c, int32_t dtype, int64_t B, int64_t n, int64_t k, int32_t d,
                         int32_t *assign_out, double *loss_out, void *stream)
{
    if (!dist_args_ok(x, c, dtype, B, n, k, d))
        return KM_ERR_INVALID;
    if (!assign_out || !loss_out) {
        set_error("distortion_fwd: null output");
        return KM_ERR_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    if (dtype == KM_F32)
        return d == 2 ? fwd_t<float, 2>((const float *)x, (const float *)c, B, n, k, assign_out, loss_out, st)
                      : fwd_t<float, 3>((const float *)x, (const float *)c, B, n, k, assign_out, loss_out, st);
    return d == 2 ? fwd_t<double, 2>((const double *)x, (const double *)c, B, n, k, assign_out, loss_out, st)
                  : fwd_t<double, 3>((const double *)x, (const double *)c, B, n, k, assign_out, loss_out, st);
}

km_status distortion_bwd(const void *x, const void *c, const int32_t *assign, const double *grad_loss, int32_t dtype,
                         int64_t B, int64_t n, int64_t k, int32_t d, void *grad_x, void *grad_c, void *stream)
{
    if (!dist_args_ok(x, c, dtype, B, n, k, d))
        return KM_ERR_INVALID;
    if (!assign || !grad_loss) {
        set_error("distortion_bwd: null assignment or grad_loss");
        return KM_ERR_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    if (dtype == KM_F32)
        return d == 2 ? bwd_alloc<float, 2>((const float *)x, (const float *)c, assign, grad_loss, B, n, k,
                                            (float *)grad_x, (float *)grad_c, st)
                      : bwd_alloc<float, 3>((const float *)x, (const float *)c, assign, grad_loss, B, n, k,
                                            (float *)grad_x, (float *)grad_c, st);
    return d == 2 ? bwd_alloc<double, 2>((const double *)x, (const double *)c, assign, grad_loss, B, n, k,
                                         (double *)grad_x, (double *)grad_c, st)
                  : bwd_alloc<double, 3>((const double *)x, (const double *)c, assign, grad_loss, B, n, k,
                                         (double *)grad_x, (double *)grad_c, st);
}

km_status distortion_bwd_noalloc(const void *x, const void *c, const int32_t *assign, const double *grad_loss,
                                 int32_t dtype, int64_t B, int64_t n, int64_t k, int32_t d, void *grad_x,
                                 void *grad_c, void *stream)
{
    if (!dist_args_ok(x, c, dtype, B, n, k, d))
        return KM_ERR_INVALID;
    if (!assign || !grad_loss) {
        set_error("distortion_bwd_noalloc: null assignment or grad_loss");
        return KM_ERR_INVALID;
    }
    if (grad_c && dist_scratch_bytes(B, k, d) > NOALLOC_SCRATCH_BYTES) {
        set_error("distortion_bwd_noalloc: B * k * (16 d + 4) bytes of cluster sums (" +
                  std::to_string(dist_scratch_bytes(B, k, d)) + " with alignment) exceed the fixed scratch of " +
                  std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes");
        return KM_ERR_INVALID;
    }
    void *buf = nullptr;
    if (grad_c) {
        km_status s = noalloc_scratch(&buf);
        if (s != KM_OK)
            return s;
    }
    hipStream_t st = (hipStream_t)stream;
    if (dtype == KM_F32)
        return d == 2 ? bwd_t<float, 2>((const float *)x, (const float *)c, assign, grad_loss, B, n, k,
                                        (float *)grad_x, (float *)grad_c, buf, st)
                      : bwd_t<float, 3>((const float *)x, (const float *)c, assign, grad_loss, B, n, k,
                                        (float *)grad_x, (float *)grad_c, buf, st);
    return d == 2 ? bwd_t<double, 2>((const double *)x, (const double *)c, assign, grad_loss, B, n, k,
                                     (double *)grad_x, (double *)grad_c, buf, st)
                  : bwd_t<double, 3>((const double *)x, (const double *)c, assign, grad_loss, B, n, k,
                                     (double *)grad_x, (double *)grad_c, buf, st);
}

} // extern "C"
