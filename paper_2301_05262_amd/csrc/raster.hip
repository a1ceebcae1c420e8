// Light-view and camera z-buffer rasteriser and per-pixel feature gather.
//
// The shadow-map pass is the vanilla rasterised depth map of paper Sec. 1 and
// 3.1 (one light-view map, no cascades); the camera pass provides the
// G-buffer (Sec. 3.1).  Both are exact: vertices are snapped to 24.8 fixed
// point, coverage uses 64-bit integer edge functions with a tie rule that
// gives shared edges to exactly one triangle, depth is interpolated in
// float64 and rounded to float32, and the nearest fragment is kept with an
// order-independent integer atomicMin.  Results are therefore identical bit
// for bit from run to run and to any other implementation of the same
// arithmetic.
//
// This file is compiled with -ffp-contract=off: every float product and sum
// below is rounded on its own, in the order written.
//
// Work distribution (MI355X): one thread per triangle sets up its snapped
// vertices and the 8x8-texel tiles its bounding box touches; a one-block scan
// turns tile counts into offsets; then every 64-lane wave rasterises one
// (triangle, tile) item at a time, one lane per texel, walking a contiguous
// run of items so that consecutive items mostly share a triangle.
#include <hip/hip_runtime.h>

#include "internal.h"

#pragma clang fp contract(off)

namespace nsm {
namespace {

constexpr uint32_t kEmptyDepth = 0x7F800000u;
constexpr unsigned long long kEmptyKey = ~0ull;
constexpr int kScanThreads = 1024;
constexpr int kRasterBlocks = 4096;   // 16384 waves: ~64 per CU on 256 CUs

__device__ __forceinline__ void to_clip(const Mat4& M, float x, float y, float z, float c[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float acc = M.m[4 * r + 0] * x;
        acc = acc + M.m[4 * r + 1] * y;
        acc = acc + M.m[4 * r + 2] * z;
        c[r] = acc + M.m[4 * r + 3];
    }
}

__device__ __forceinline__ int64_t floor_div256(int64_t a) {
    return (a >= 0) ? (a >> 8) : -((-a + 255) >> 8);
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_tri_setup(const float* __restrict__ tris, int n_tris, Mat4 M, int w, int h,
                            TriSetup* __restrict__ setup, int* __restrict__ counts) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tris) return;
    const float* T = tris + 9 * (size_t)t;
    const float fw = (float)w, fh = (float)h;
    int64_t X[3], Y[3];
    float Z[3];
    bool drop = false;
    for (int v = 0; v < 3; ++v) {
        float c[4];
        to_clip(M, T[3 * v], T[3 * v + 1], T[3 * v + 2], c);
        if (!(c[3] > 1e-6f)) { drop = true; break; }
        float nx = c[0] / c[3];
        float ny = c[1] / c[3];
        float nz = c[2] / c[3];
        float sx = (nx * 0.5f + 0.5f) * fw;
        float sy = (ny * 0.5f + 0.5f) * fh;
        if (!(sx >= -8.0f * fw && sx <= 9.0f * fw && sy >= -8.0f * fh && sy <= 9.0f * fh)) {
            drop = true;
            break;
        }
        X[v] = (int64_t)rintf(sx * 256.0f);
        Y[v] = (int64_t)rintf(sy * 256.0f);
        Z[v] = nz;
    }
    int count = 0;
    TriSetup s;
    s.pad = 0;
    if (!drop) {
        int64_t A = (X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]);
        if (A != 0) {
            if (A < 0) {  // make the vertex order counter-clockwise (no culling)
                int64_t tx = X[1]; X[1] = X[2]; X[2] = tx;
                int64_t ty = Y[1]; Y[1] = Y[2]; Y[2] = ty;
                float tz = Z[1]; Z[1] = Z[2]; Z[2] = tz;
                A = -A;
            }
            int64_t xmin = min(X[0], min(X[1], X[2])), xmax = max(X[0], max(X[1], X[2]));
            int64_t ymin = min(Y[0], min(Y[1], Y[2])), ymax = max(Y[0], max(Y[1], Y[2]));
            int64_t i0 = max((int64_t)0, floor_div256(xmin - 128));
            int64_t i1 = min((int64_t)(w - 1), floor_div256(xmax - 128) + 1);
            int64_t j0 = max((int64_t)0, floor_div256(ymin - 128));
            int64_t j1 = min((int64_t)(h - 1), floor_div256(ymax - 128) + 1);
            if (i0 <= i1 && j0 <= j1) {
                int tx0 = (int)(i0 >> 3), tx1 = (int)(i1 >> 3);
                int ty0 = (int)(j0 >> 3), ty1 = (int)(j1 >> 3);
                s.tx0 = tx0;
                s.ty0 = ty0;
                s.ntx = tx1 - tx0 + 1;
                count = s.ntx * (ty1 - ty0 + 1);
            }
            for (int v = 0; v < 3; ++v) {
                s.x[v] = (int32_t)X[v];
                s.y[v] = (int32_t)Y[v];
                s.z[v] = Z[v];
            }
            s.area = A;
        }
    }
    if (count == 0) {
        s.tx0 = s.ty0 = 0;
        s.ntx = 1;
        s.area = 0;
        for (int v = 0; v < 3; ++v) { s.x[v] = 0; s.y[v] = 0; s.z[v] = 0.0f; }
    }
    setup[t] = s;
    counts[t] = count;
}

// Exclusive scan of counts[0..n) into offsets[0..n] (offsets[n] = total), one block.
__global__ void __launch_bounds__(kScanThreads) k_scan(const int* __restrict__ counts, int n,
                                                       long long* __restrict__ offsets) {
    __shared__ long long part[kScanThreads];
    int tid = threadIdx.x;
    int chunk = (n + kScanThreads - 1) / kScanThreads;
    int b = tid * chunk, e = min(n, b + chunk);
    long long sum = 0;
    for (int i = b; i < e; ++i) sum += counts[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {   // Hillis-Steele inclusive scan
        long long v = (tid >= off) ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    long long run = part[tid] - sum;
    for (int i = b; i < e; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (tid == kScanThreads - 1) offsets[n] = part[tid];
}

__device__ __forceinline__ bool edge_inclusive(int64_t dx, int64_t dy) {
    return dy > 0 || (dy == 0 && dx < 0);
}

template <bool KEY64>
__global__ void __launch_bounds__(256) k_raster(const TriSetup* __restrict__ setup,
                                                const long long* __restrict__ offsets, int n_tris,
                                                int w, int h, void* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const long long wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const long long nwaves = gridDim.x * (blockDim.x >> 6);
    const long long total = offsets[n_tris];
    const long long per = (total + nwaves - 1) / nwaves;
    const long long begin = wave * per;
    const long long end = min(total, begin + per);
    if (begin >= end) return;
    // largest t with offsets[t] <= begin
    int lo = 0, hi = n_tris;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (offsets[mid] <= begin) lo = mid; else hi = mid;
    }
    int t = lo;
    for (long long item = begin; item < end; ++item) {
        while (offsets[t + 1] <= item) ++t;
        const TriSetup s = setup[t];
        const int local = (int)(item - offsets[t]);
        const int tx = s.tx0 + local % s.ntx;
        const int ty = s.ty0 + local / s.ntx;
        const int i = tx * 8 + (lane & 7);
        const int j = ty * 8 + (lane >> 3);
        if (i >= w || j >= h) continue;
        const int64_t px = 256 * (int64_t)i + 128, py = 256 * (int64_t)j + 128;
        const int64_t X0 = s.x[0], X1 = s.x[1], X2 = s.x[2];
        const int64_t Y0 = s.y[0], Y1 = s.y[1], Y2 = s.y[2];
        // E_k: edge opposite vertex k, positive inside a CCW triangle
        const int64_t e0 = (X2 - X1) * (py - Y1) - (Y2 - Y1) * (px - X1);
        const int64_t e1 = (X0 - X2) * (py - Y2) - (Y0 - Y2) * (px - X2);
        const int64_t e2 = (X1 - X0) * (py - Y0) - (Y1 - Y0) * (px - X0);
        const bool in0 = e0 > 0 || (e0 == 0 && edge_inclusive(X2 - X1, Y2 - Y1));
        const bool in1 = e1 > 0 || (e1 == 0 && edge_inclusive(X0 - X2, Y0 - Y2));
        const bool in2 = e2 > 0 || (e2 == 0 && edge_inclusive(X1 - X0, Y1 - Y0));
        if (!(in0 && in1 && in2)) continue;
        double num = (double)e0 * (double)s.z[0];
        num = num + (double)e1 * (double)s.z[1];
        num = num + (double)e2 * (double)s.z[2];
        const float d = (float)(num / (double)s.area);
        if (!(d >= 0.0f && d <= 1.0f)) continue;
        uint32_t bits = __float_as_uint(d);
        if ((bits & 0x7FFFFFFFu) == 0) bits = 0;  // -0 -> +0
        const size_t k = (size_t)j * (size_t)w + (size_t)i;
        if (KEY64) {
            unsigned long long key = ((unsigned long long)bits << 32) | (unsigned long long)(uint32_t)t;
            atomicMin(reinterpret_cast<unsigned long long*>(out) + k, key);
        } else {
            atomicMin(reinterpret_cast<uint32_t*>(out) + k, bits);
        }
    }
}

__device__ __forceinline__ float lin_depth(float q, float nl, float fl) {
    float num = nl * fl;
    float den = fl - q * (fl - nl);
    return num / den;
}

template <bool SOFT>
__global__ void __launch_bounds__(256) k_gather(const float* __restrict__ tris,
                                                const float* __restrict__ normals, int n_tris,
                                                GatherParams P,
                                                const unsigned long long* __restrict__ gbuf,
                                                const uint32_t* __restrict__ sm, int w, int h,
                                                float* __restrict__ feat, uint8_t* __restrict__ mask) {
    constexpr int C = SOFT ? 8 : 6;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= w) return;
    const size_t p = (size_t)j * (size_t)w + (size_t)i;
    float f[C];
#pragma unroll
    for (int c = 0; c < C; ++c) f[c] = 0.0f;
    uint8_t mk = 0;
    const unsigned long long key = gbuf[p];
    const uint32_t t = (uint32_t)(key & 0xFFFFFFFFull);
    bool fg = key != kEmptyKey && (int)t < n_tris;
    double D[3], tt = 0.0;
    if (fg) {
        // receiver: the pixel-centre camera ray meets the triangle's plane (float64)
        const double ndcx = (2.0 * ((double)i + 0.5)) / (double)w - 1.0;
        const double ndcy = (2.0 * ((double)j + 0.5)) / (double)h - 1.0;
        const double ax = ndcx * (double)P.tanx, ay = ndcy * (double)P.tany;
#pragma unroll
        for (int k = 0; k < 3; ++k) D[k] = ((double)P.fwd[k] + ax * (double)P.right[k]) + ay * (double)P.up[k];
        const float* V0 = tris + 9 * (size_t)t;
        const float* N = normals + 3 * (size_t)t;
        double num = (double)N[0] * ((double)V0[0] - (double)P.E[0]);
        num = num + (double)N[1] * ((double)V0[1] - (double)P.E[1]);
        num = num + (double)N[2] * ((double)V0[2] - (double)P.E[2]);
        double den = (double)N[0] * D[0];
        den = den + (double)N[1] * D[1];
        den = den + (double)N[2] * D[2];
        if (den == 0.0) fg = false;
        else tt = num / den;
    }
    if (fg) {
        const float* N = normals + 3 * (size_t)t;
        float Pw[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) Pw[k] = (float)((double)P.E[k] + tt * D[k]);
        float n0 = N[0], n1 = N[1], n2 = N[2];
        const float vx = P.E[0] - Pw[0], vy = P.E[1] - Pw[1], vz = P.E[2] - Pw[2];
        float sgn = n0 * vx + n1 * vy;
        sgn = sgn + n2 * vz;
        if (sgn < 0.0f) { n0 = -n0; n1 = -n1; n2 = -n2; }
        float dv = (Pw[0] - P.E[0]) * P.fwd[0] + (Pw[1] - P.E[1]) * P.fwd[1];
        dv = dv + (Pw[2] - P.E[2]) * P.fwd[2];
        float c[4];
        to_clip(P.ml, Pw[0], Pw[1], Pw[2], c);
        bool inside = c[3] > 1e-6f;
        float zf = P.fl, z = P.fl;
        int ti = 0, tj = 0;
        if (inside) {
            const float nx = c[0] / c[3], ny = c[1] / c[3], nz = c[2] / c[3];
            const float sx = (nx * 0.5f + 0.5f) * (float)P.S;
            const float sy = (ny * 0.5f + 0.5f) * (float)P.S;
            zf = lin_depth(nz, P.nl, P.fl);
            inside = sx >= 0.0f && sx < (float)P.S && sy >= 0.0f && sy < (float)P.S && nz >= 0.0f &&
                     nz <= 1.0f;
            if (inside) {
                ti = (int)floorf(sx);
                tj = (int)floorf(sy);
                const uint32_t b = sm[(size_t)tj * (size_t)P.S + (size_t)ti];
                if (b == kEmptyDepth) inside = false;
                else z = lin_depth(__uint_as_float(b), P.nl, P.fl);
            }
        }
        // slope-scaled depth bias from the angle between normal and light direction
        const float tau = (2.0f * P.tanl) / (float)P.S;
        const float lx = P.L[0] - Pw[0], ly = P.L[1] - Pw[1], lz = P.L[2] - Pw[2];
        float ll = lx * lx + ly * ly;
        ll = ll + lz * lz;
        const float len = sqrtf(ll);
        const float hx = lx / len, hy = ly / len, hz = lz / len;
        float cl = n0 * hx + n1 * hy;
        cl = cl + n2 * hz;
        const float sn = sqrtf(fmaxf(1.0f - cl * cl, 0.0f));
        const float tq = sn / fmaxf(cl, 1e-3f);
        const float beta = (zf * tau) * (1.0f + 1.5f * fminf(tq, 10.0f));
        mk = (inside && zf > z + beta) ? 1 : 0;
        f[0] = dv / P.fc;
        f[1] = n0;
        f[2] = n1;
        f[3] = n2;
        f[4] = (z - zf) / P.fl;
        f[5] = z / P.fl;
        if (SOFT) {
            float zb = zf;
            if (inside) {
                const float thr = zf - beta;
                float sum = 0.0f;
                int cnt = 0;
                for (int dj = -3; dj <= 3; ++dj) {
                    const int jj = tj + dj;
                    if (jj < 0 || jj >= P.S) continue;
                    for (int di = -3; di <= 3; ++di) {
                        const int ii = ti + di;
                        if (ii < 0 || ii >= P.S) continue;
                        const uint32_t b = sm[(size_t)jj * (size_t)P.S + (size_t)ii];
                        if (b == kEmptyDepth) continue;
                        const float q = lin_depth(__uint_as_float(b), P.nl, P.fl);
                        if (q < thr) { sum = sum + q; ++cnt; }
                    }
                }
                if (cnt > 0) zb = sum / (float)cnt;
            }
            f[C - 2] = P.r_e / 0.2f;
            f[C - 1] = zb / P.fl;
        }
    }
    float* o = feat + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) o[c] = f[c];
    if (mask) mask[p] = mk;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t raster_workspace_bytes(int n_tris) {
    return align256((size_t)n_tris * sizeof(TriSetup)) + align256((size_t)n_tris * 4) +
           align256(((size_t)n_tris + 1) * 8);
}

hipError_t raster(const float* tris, int n_tris, const Mat4& m, int w, int h, bool key64,
                  void* out, void* ws, hipStream_t s) {
    const size_t npix = (size_t)w * (size_t)h;
    const int fill_blocks = (int)min((size_t)4096, (npix + 255) / 256);
    const char* sfx = key64 ? " camera" : " light";
    {
        TraceScope ts("clear", sfx, s);
        if (key64)
            k_fill_u64<<<fill_blocks, 256, 0, s>>>(reinterpret_cast<unsigned long long*>(out), npix, kEmptyKey);
        else
            k_fill_u32<<<fill_blocks, 256, 0, s>>>(reinterpret_cast<uint32_t*>(out), npix, kEmptyDepth);
    }
    if (n_tris == 0) return hipGetLastError();
    char* base = reinterpret_cast<char*>(ws);
    TriSetup* setup = reinterpret_cast<TriSetup*>(base);
    int* counts = reinterpret_cast<int*>(base + align256((size_t)n_tris * sizeof(TriSetup)));
    long long* offsets =
        reinterpret_cast<long long*>(reinterpret_cast<char*>(counts) + align256((size_t)n_tris * 4));
    {
        TraceScope ts("tri_setup", sfx, s);
        k_tri_setup<<<(n_tris + 255) / 256, 256, 0, s>>>(tris, n_tris, m, w, h, setup, counts);
    }
    {
        TraceScope ts("tile_scan", sfx, s);
        k_scan<<<1, kScanThreads, 0, s>>>(counts, n_tris, offsets);
    }
    {
        TraceScope ts("raster", sfx, s);
        if (key64)
            k_raster<true><<<kRasterBlocks, 256, 0, s>>>(setup, offsets, n_tris, w, h, out);
        else
            k_raster<false><<<kRasterBlocks, 256, 0, s>>>(setup, offsets, n_tris, w, h, out);
    }
    return hipGetLastError();
}

hipError_t gather(const float* tris, const float* normals, int n_tris, const GatherParams& p,
                  const uint64_t* gbuf, const uint32_t* sm, int w, int h, bool soft, float* feat,
                  uint8_t* mask, hipStream_t s) {
    dim3 grid((w + 255) / 256, h);
    const auto* g = reinterpret_cast<const unsigned long long*>(gbuf);
    TraceScope ts("gather", soft ? " soft8" : " hard6", s);
    if (soft)
        k_gather<true><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, w, h, feat, mask);
    else
        k_gather<false><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, w, h, feat, mask);
    return hipGetLastError();
}

}  // namespace nsm
