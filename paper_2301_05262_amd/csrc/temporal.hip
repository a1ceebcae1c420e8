// Temporal-stability kernels.
//
// Perturbation loss (Sec. 3.3, Eq. 2), per-pixel L1 term: for each sample n,
// x_0 is the output on the unperturbed input, x_1..x_p on perturbed inputs,
// x~ the target:
//     loss = alpha / (N H W) * sum_{n, px} ( |x_0 - x~| + sum_i |x_0 - x_i| ),
//     dloss/dx_0 = alpha / (N H W) * ( sgn(x_0 - x~) + sum_i sgn(x_0 - x_i) ),
// with x_1..x_p held constant (the gradient flows through x_0 only) and
// sgn(0) = 0.  Differences and the loss sum are taken in float64.
//
// Temporal instability (Sec. 3.4, Eq. 3), one pair of consecutive frames:
// for every pixel p of the current frame with a receiver, m(p) is the pixel
// of the previous frame its surface point projects to (the motion-vector
// lookup of a static scene); pixels off-screen, on an empty previous pixel,
// or failing the depth (relative view depth along the previous camera) or
// normal (cosine) comparison are rejected; the others add
// exp(alpha |I_t(p) - I_{t-1}(m(p))|) - 1 (float64).
//
// Both reductions are deterministic: per-block float64 partials, then one
// block sums them in a fixed order.  This file is compiled without
// floating-point contraction so that the receiver reconstruction and the
// projection round every product and sum in the written order (the
// decisions that depend on them are exact).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

#pragma clang fp contract(off)

namespace nsm {
namespace {

constexpr int kThreadsT = 256;
constexpr unsigned long long kEmptyKeyT = ~0ull;

// Sum of one float64 per thread of a 256-thread block, in a fixed order;
// the result is valid in thread 0.
__device__ double block_sum256(double v, double* sh) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kThreadsT)
    k_perturb_loss(const float* __restrict__ vis, const float* __restrict__ target, int p, long long hw,
                   long long total, double scale, float* __restrict__ dvis0, double* __restrict__ partials) {
    __shared__ double sh[4];
    const long long idx = (long long)blockIdx.x * kThreadsT + threadIdx.x;
    double acc = 0.0;
    if (idx < total) {
        const long long f = idx / hw, q = idx - f * hw;
        const float* v = vis + f * (long long)(1 + p) * hw + q;
        const double x0 = (double)v[0];
        const double dt = x0 - (double)target[idx];
        acc = fabs(dt);
        double g = (dt > 0.0) - (dt < 0.0);
        for (int i = 1; i <= p; ++i) {
            const double d = x0 - (double)v[(long long)i * hw];
            acc += fabs(d);
            g += (d > 0.0) - (d < 0.0);
        }
        dvis0[idx] = (float)(scale * g);
    }
    const double s = block_sum256(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[c] = (accumulate ? out[c] : 0) + scale * sum_b partials[b * ncomp + c]
__global__ void __launch_bounds__(kThreadsT)
    k_reduce_partials(const double* __restrict__ partials, int nblk, int ncomp, double scale,
                      double* __restrict__ out, int accumulate) {
    __shared__ double sh[4];
    for (int c = 0; c < ncomp; ++c) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kThreadsT) v += partials[(size_t)b * ncomp + c];
        const double s = block_sum256(v, sh);
        if (threadIdx.x == 0) out[c] = (accumulate ? out[c] : 0.0) + scale * s;
    }
}

__device__ __forceinline__ void clip4(const float* M, const float P[3], float c[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float acc = M[4 * r + 0] * P[0];
        acc = acc + M[4 * r + 1] * P[1];
        acc = acc + M[4 * r + 2] * P[2];
        c[r] = acc + M[4 * r + 3];
    }
}

// Receiver of pixel (i, j): the pixel-centre camera ray meets the plane of
// the key's triangle (float64, rounded to float32); normal flipped towards
// the camera.  False for background and degenerate rays.
__device__ bool receiver(const float* __restrict__ tris, const float* __restrict__ normals, int n_tris,
                         const CamParams& c, unsigned long long key, int i, int j, int w, int h, float P[3],
                         float n[3]) {
    if (key == kEmptyKeyT) return false;
    const uint32_t t = (uint32_t)(key & 0xFFFFFFFFull);
    if ((int)t >= n_tris) return false;
    const double ndcx = (2.0 * ((double)i + 0.5)) / (double)w - 1.0;
    const double ndcy = (2.0 * ((double)j + 0.5)) / (double)h - 1.0;
    const double ax = ndcx * (double)c.tanx, ay = ndcy * (double)c.tany;
    double D[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) D[k] = ((double)c.fwd[k] + ax * (double)c.right[k]) + ay * (double)c.up[k];
    const float* V0 = tris + 9 * (size_t)t;
    const float* N = normals + 3 * (size_t)t;
    double num = (double)N[0] * ((double)V0[0] - (double)c.E[0]);
    num = num + (double)N[1] * ((double)V0[1] - (double)c.E[1]);
    num = num + (double)N[2] * ((double)V0[2] - (double)c.E[2]);
    double den = (double)N[0] * D[0];
    den = den + (double)N[1] * D[1];
    den = den + (double)N[2] * D[2];
    if (den == 0.0) return false;
    const double tt = num / den;
#pragma unroll
    for (int k = 0; k < 3; ++k) P[k] = (float)((double)c.E[k] + tt * D[k]);
    n[0] = N[0];
    n[1] = N[1];
    n[2] = N[2];
    const float vx = c.E[0] - P[0], vy = c.E[1] - P[1], vz = c.E[2] - P[2];
    float s = n[0] * vx + n[1] * vy;
    s = s + n[2] * vz;
    if (s < 0.0f) {
        n[0] = -n[0];
        n[1] = -n[1];
        n[2] = -n[2];
    }
    return true;
}

__device__ __forceinline__ float view_depth(const CamParams& c, const float P[3]) {
    const float dv = (P[0] - c.E[0]) * c.fwd[0] + (P[1] - c.E[1]) * c.fwd[1];
    return dv + (P[2] - c.E[2]) * c.fwd[2];
}

__global__ void __launch_bounds__(kThreadsT)
    k_temporal(const float* __restrict__ tris, const float* __restrict__ normals, int n_tris, CamParams prev,
               CamParams cur, const unsigned long long* __restrict__ gprev,
               const unsigned long long* __restrict__ gcur, const float* __restrict__ vprev,
               const float* __restrict__ vcur, int w, int h, float alpha, float depth_tol, float cos_tol,
               float* __restrict__ d_out, double* __restrict__ partials) {
    __shared__ double sh[4];
    const long long idx = (long long)blockIdx.x * kThreadsT + threadIdx.x;
    double term = 0.0, passed = 0.0;
    if (idx < (long long)w * h) {
        const int j = (int)(idx / w), i = (int)(idx - (long long)j * w);
        float code = -1.0f;
        float P[3], n[3];
        if (receiver(tris, normals, n_tris, cur, gcur[idx], i, j, w, h, P, n)) {
            float c[4];
            clip4(prev.m, P, c);
            code = -2.0f;
            if (c[3] > 1e-6f) {
                const float nx = c[0] / c[3], ny = c[1] / c[3];
                const float sx = (nx * 0.5f + 0.5f) * (float)w;
                const float sy = (ny * 0.5f + 0.5f) * (float)h;
                if (sx >= 0.0f && sx < (float)w && sy >= 0.0f && sy < (float)h) {
                    const int iq = (int)floorf(sx), jq = (int)floorf(sy);
                    const size_t q = (size_t)jq * (size_t)w + (size_t)iq;
                    float Pq[3], nq[3];
                    code = -3.0f;
                    if (receiver(tris, normals, n_tris, prev, gprev[q], iq, jq, w, h, Pq, nq)) {
                        const float dv = view_depth(prev, P), dq = view_depth(prev, Pq);
                        float cs = n[0] * nq[0] + n[1] * nq[1];
                        cs = cs + n[2] * nq[2];
                        if (fabsf(dv - dq) > depth_tol * dq) {
                            code = -4.0f;
                        } else if (cs < cos_tol) {
                            code = -5.0f;
                        } else {
                            const float D = fabsf(vcur[idx] - vprev[q]);
                            term = exp((double)alpha * (double)D) - 1.0;
                            passed = 1.0;
                            code = D;
                        }
                    }
                }
            }
        }
        if (d_out) d_out[idx] = code;
    }
    const double s = block_sum256(term, sh);
    const double k = block_sum256(passed, sh);
    if (threadIdx.x == 0) {
        partials[2 * (size_t)blockIdx.x] = s;
        partials[2 * (size_t)blockIdx.x + 1] = k;
    }
}

}  // namespace

// Scratch of the allocation-free perturbation-loss entry point: the per-block
// float64 partial sums (one per 256 pixels), held by each device the library
// runs on until the process ends.  In host code `scratch` names a host-side
// stand-in; kernels get the device address from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kStaticLossPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_loss_partials(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        // the current device's copy of the array (each device holds its own)
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t perturb_loss_workspace_bytes(long long npx) {
    const long long nblk = (npx + kThreadsT - 1) / kThreadsT;
    return (size_t)(nblk > 0 ? nblk : 1) * sizeof(double);
}

hipError_t perturb_loss(const float* vis, const float* target, int n, int p, int h, int w, float alpha,
                        double* loss, float* dvis0, void* ws, hipStream_t s) {
    const long long hw = (long long)h * w, total = (long long)n * hw;
    const int nblk = (int)((total + kThreadsT - 1) / kThreadsT);
    double* partials = reinterpret_cast<double*>(ws);
    const double scale = (double)alpha / (double)total;
    TraceScope ts("perturbation loss", "", s);
    k_perturb_loss<<<nblk, kThreadsT, 0, s>>>(vis, target, p, hw, total, scale, dvis0, partials);
    k_reduce_partials<<<1, kThreadsT, 0, s>>>(partials, nblk, 1, scale, loss, 0);
    return hipGetLastError();
}

size_t temporal_workspace_bytes(int h, int w) {
    const long long nblk = ((long long)h * w + kThreadsT - 1) / kThreadsT;
    return (size_t)(nblk > 0 ? nblk : 1) * 2 * sizeof(double);
}

hipError_t temporal_pair(const float* tris, const float* normals, int n_tris, const CamParams& prev,
                         const CamParams& cur, const uint64_t* gprev, const uint64_t* gcur, const float* vprev,
                         const float* vcur, int h, int w, float alpha, float depth_tol, float cos_tol,
                         int accumulate, double* acc_out, float* d_out, void* ws, hipStream_t s) {
    const int nblk = (int)(((long long)h * w + kThreadsT - 1) / kThreadsT);
    double* partials = reinterpret_cast<double*>(ws);
    TraceScope ts("temporal instability", "", s);
    k_temporal<<<nblk, kThreadsT, 0, s>>>(tris, normals, n_tris, prev, cur,
                                          reinterpret_cast<const unsigned long long*>(gprev),
                                          reinterpret_cast<const unsigned long long*>(gcur), vprev, vcur, w, h,
                                          alpha, depth_tol, cos_tol, d_out, partials);
    k_reduce_partials<<<1, kThreadsT, 0, s>>>(partials, nblk, 2, 1.0, acc_out, accumulate);
    return hipGetLastError();
}

}  // namespace nsm
