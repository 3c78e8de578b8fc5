// Measurement kernels (librowbench.so): streaming reads for the achievable
// HBM bandwidth, and sorted-row intersections |N(u) & N(v)| over row pairs
// with four variants of the set operation (Sec. 4.1, Sec. 5.1).  Not part
// of the matching path; they time the operation the engine is made of.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <string>

#include "../../include/rowbench.h"

namespace {

thread_local std::string g_err;

constexpr int kP = 64;          // pairs per wavefront in the batched variants
constexpr int kLdsInts = 4096;  // LDS staging capacity of RB_LDS (16 KB)

__device__ __forceinline__ int wave_scan_excl(int x, int lane, int *tot) {
    int inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    *tot = __shfl(inc, 63, 64);
    return inc - x;
}

// first index in [lo, hi) with a[i] >= key (hi if none)
template <class T>
__device__ __forceinline__ int lower_bound(const T *a, int lo, int hi, int32_t key) {
    int n = hi - lo;
    while (n > 0) {
        const int half = n >> 1;
        if (a[lo + half] < key) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo;
}

__global__ void __launch_bounds__(256) stream_read_kernel(const uint4 *__restrict__ p, long long n4,
                                                          unsigned long long *sum) {
    unsigned long long acc = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
        acc += (unsigned long long)a.x + a.y + a.z + a.w;
        acc += (unsigned long long)b.x + b.y + b.z + b.w;
        acc += (unsigned long long)c.x + c.y + c.z + c.w;
        acc += (unsigned long long)d.x + d.y + d.z + d.w;
    }
    for (; i < n4; i += stride) {
        const uint4 a = p[i];
        acc += (unsigned long long)a.x + a.y + a.z + a.w;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(sum, acc);
}

__global__ void __launch_bounds__(256) fill_kernel(uint4 *p, long long n4, uint32_t v) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) p[i] = make_uint4(v, v, v, v);
}

// The batched variants: a wavefront takes 64 pairs, lane l sets up pair l
// (A = its shorter row, B = the longer), the A rows are laid end to end by
// a wave scan, and lane t walks elements t, t + 64, ... of that
// concatenation with a monotone segment cursor, testing each in its pair's
// B; per-pair counts gather in LDS.
template <int kVariant>
__global__ void __launch_bounds__(64) isect_batched(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ pu, const int32_t *__restrict__ pv,
                                                    long long np, uint32_t *__restrict__ out) {
    __shared__ int32_t seg_start[kP + 1];
    __shared__ long long sa[kP], sb[kP];
    __shared__ int32_t slb[kP], sbl[kP];
    __shared__ uint32_t cnt[kP];
    __shared__ int32_t lds_b[kVariant == RB_LDS ? kLdsInts : 1];
    const int lane = threadIdx.x;
    for (long long base = (long long)blockIdx.x * kP; base < np; base += (long long)gridDim.x * kP) {
        const int n = (int)min((long long)kP, np - base);
        long long a0 = 0, b0 = 0;
        int la = 0, lb = 0;
        if (lane < n) {
            const int32_t u = pu[base + lane], v = pv[base + lane];
            const long long su = rp[u], sv = rp[v];
            const int lu = (int)(rp[u + 1] - su), lv = (int)(rp[v + 1] - sv);
            if (lu <= lv) {
                a0 = su, la = lu, b0 = sv, lb = lv;
            } else {
                a0 = sv, la = lv, b0 = su, lb = lu;
            }
        }
        int tot = 0;
        const int st = wave_scan_excl(la, lane, &tot);
        seg_start[lane] = st;
        if (lane == 0) seg_start[kP] = tot;
        sa[lane] = a0;
        sb[lane] = b0;
        slb[lane] = lb;
        cnt[lane] = 0;
        bool staged = false;
        if constexpr (kVariant == RB_LDS) {
            int totb = 0;
            sbl[lane] = wave_scan_excl(lb, lane, &totb);
            staged = totb <= kLdsInts;
            __syncthreads();
            if (staged) {
                // each B row copied by the whole wavefront, lanes on
                // consecutive elements (coalesced)
                for (int s = 0; s < n; s++) {
                    const int len = slb[s], dst = sbl[s];
                    const int32_t *src = col + sb[s];
                    for (int j = lane; j < len; j += 64) lds_b[dst + j] = src[j];
                }
            }
        }
        __syncthreads();
        int s = 0;
        int gseg = -1, gpos = 0;  // RB_GALLOP: where this lane's last element of segment gseg landed
        for (int tb = 0; tb < tot; tb += 64) {
            const int t = tb + lane;
            bool found = false;
            if (t < tot) {
                while (seg_start[s + 1] <= t) s++;
                const int32_t key = col[sa[s] + (t - seg_start[s])];
                const int lbs = slb[s];
                if (kVariant == RB_LDS && staged) {
                    const int32_t *B = lds_b + sbl[s];
                    const int i = lower_bound(B, 0, lbs, key);
                    found = i < lbs && B[i] == key;
                } else if (kVariant == RB_GALLOP) {
                    const int32_t *B = col + sb[s];
                    if (s != gseg) {
                        gseg = s;
                        gpos = 0;
                    }
                    // exponential steps from the last landing point, then a
                    // binary search inside the last step
                    int lo = gpos, hi = gpos, step = 1;
                    while (hi < lbs && B[hi] < key) {
                        lo = hi + 1;
                        hi = lo + step;
                        step <<= 1;
                    }
                    if (hi > lbs) hi = lbs;
                    const int i = lower_bound(B, lo, hi, key);
                    gpos = i;
                    found = i < lbs && B[i] == key;
                } else {
                    const int32_t *B = col + sb[s];
                    const int i = lower_bound(B, 0, lbs, key);
                    found = i < lbs && B[i] == key;
                }
            }
            if (found) atomicAdd(&cnt[s], 1u);
        }
        __syncthreads();
        if (lane < n) out[base + lane] = cnt[lane];
        __syncthreads();
    }
}

// One wavefront per pair: the merge of A and B (ties: A first) is cut into
// 64 diagonals of equal length; a lane finds where its diagonal crosses
// the merge by a binary search, then merges its part.  An element of A is
// in B exactly when, at the moment it is consumed, the smallest unconsumed
// element of B equals it, so no pair is missed at a cut.
__global__ void __launch_bounds__(64) isect_mergepath(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                      const int32_t *__restrict__ pu, const int32_t *__restrict__ pv,
                                                      long long np, uint32_t *__restrict__ out) {
    const int lane = threadIdx.x;
    for (long long p = blockIdx.x; p < np; p += gridDim.x) {
        const int32_t u = pu[p], v = pv[p];
        const int32_t *A = col + rp[u];
        const int32_t *B = col + rp[v];
        const int la = (int)(rp[u + 1] - rp[u]), lb = (int)(rp[v + 1] - rp[v]);
        const int total = la + lb;
        const int per = (total + 63) / 64;
        const int d0 = min(lane * per, total), d1 = min(d0 + per, total);
        int lo = max(0, d0 - lb), hi = min(d0, la);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A[mid] <= B[d0 - 1 - mid]) lo = mid + 1;
            else hi = mid;
        }
        int i = lo, j = d0 - lo;
        int32_t a = i < la ? A[i] : INT_MAX, b = j < lb ? B[j] : INT_MAX;
        uint32_t c = 0;
        for (int d = d0; d < d1; d++) {
            if (i < la && (j >= lb || a <= b)) {
                c += (j < lb && a == b) ? 1u : 0u;
                i++;
                a = i < la ? A[i] : INT_MAX;
            } else {
                j++;
                b = j < lb ? B[j] : INT_MAX;
            }
        }
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
        if (lane == 0) out[p] = c;
    }
}

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define RB_CK(call)                                                                   \
    do {                                                                              \
        const hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) return fail(-3, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" {

const char *rb_last_error(void) { return g_err.c_str(); }

int rb_stream_read(const void *buf, int64_t n_words, int32_t reps, uint64_t *acc, double *ms_per_pass,
                   uint64_t *checksum, void *hip_stream) {
    if (!buf || !acc || n_words <= 0 || n_words % 4 || reps < 1 || !ms_per_pass || !checksum ||
        reinterpret_cast<uintptr_t>(buf) % 16)
        return fail(-1, "bad arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(-3, "device query failed");
    unsigned long long *a = reinterpret_cast<unsigned long long *>(acc);
    hipEvent_t e0, e1;
    RB_CK(hipEventCreate(&e0));
    RB_CK(hipEventCreate(&e1));
    RB_CK(hipMemsetAsync(a, 0, sizeof(unsigned long long), s));
    const long long n4 = n_words / 4;
    const int grid = ncu * 8;
    // one untimed pass first
    hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(256), 0, s, static_cast<const uint4 *>(buf), n4, a);
    RB_CK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; r++)
        hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(256), 0, s, static_cast<const uint4 *>(buf), n4, a);
    RB_CK(hipEventRecord(e1, s));
    unsigned long long h = 0;
    RB_CK(hipMemcpyAsync(&h, a, sizeof(h), hipMemcpyDeviceToHost, s));
    const hipError_t e = hipStreamSynchronize(s);
    float ms = 0.f;
    RB_CK(hipEventElapsedTime(&ms, e0, e1));
    RB_CK(hipEventDestroy(e0));
    RB_CK(hipEventDestroy(e1));
    if (e != hipSuccess) return fail(-3, std::string("stream read: ") + hipGetErrorString(e));
    *ms_per_pass = (double)ms / reps;
    *checksum = h;
    return 0;
}

int rb_flush(void *buf, int64_t n_words, void *hip_stream) {
    if (!buf || n_words <= 0 || n_words % 4 || reinterpret_cast<uintptr_t>(buf) % 16) return fail(-1, "bad arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    static uint32_t v = 1;
    hipLaunchKernelGGL(fill_kernel, dim3(4096), dim3(256), 0, s, static_cast<uint4 *>(buf), n_words / 4, v++);
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(-3, std::string("flush: ") + hipGetErrorString(e));
    return 0;
}

int rb_intersect(int32_t variant, const int64_t *row_ptr, const int32_t *col, const int32_t *pu, const int32_t *pv,
                 int64_t n_pairs, uint32_t *out, int32_t grid, double *ms, void *hip_stream) {
    if (!row_ptr || !col || !pu || !pv || !out || !ms || n_pairs <= 0 || grid < 0 || variant < RB_BINARY ||
        variant > RB_LDS)
        return fail(-1, "bad arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int g = grid ? grid : 2048;
    hipEvent_t e0, e1;
    RB_CK(hipEventCreate(&e0));
    RB_CK(hipEventCreate(&e1));
    RB_CK(hipEventRecord(e0, s));
    switch (variant) {
    case RB_BINARY:
        hipLaunchKernelGGL(isect_batched<RB_BINARY>, dim3(g), dim3(64), 0, s, row_ptr, col, pu, pv, (long long)n_pairs, out);
        break;
    case RB_GALLOP:
        hipLaunchKernelGGL(isect_batched<RB_GALLOP>, dim3(g), dim3(64), 0, s, row_ptr, col, pu, pv, (long long)n_pairs, out);
        break;
    case RB_LDS:
        hipLaunchKernelGGL(isect_batched<RB_LDS>, dim3(g), dim3(64), 0, s, row_ptr, col, pu, pv, (long long)n_pairs, out);
        break;
    default:
        hipLaunchKernelGGL(isect_mergepath, dim3(g), dim3(64), 0, s, row_ptr, col, pu, pv, (long long)n_pairs, out);
    }
    RB_CK(hipEventRecord(e1, s));
    const hipError_t e = hipStreamSynchronize(s);
    float t = 0.f;
    RB_CK(hipEventElapsedTime(&t, e0, e1));
    RB_CK(hipEventDestroy(e0));
    RB_CK(hipEventDestroy(e1));
    if (e != hipSuccess) return fail(-3, std::string("intersect: ") + hipGetErrorString(e));
    *ms = t;
    return 0;
}

}  // extern "C"
