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
// vertices and the 16x4-texel tiles its bounding box touches; a one-block scan
// turns tile counts into offsets; then every 64-lane wave rasterises 64
// (triangle, tile) items at a time, runs of 4 consecutive items dealt to the
// waves in turn, one lane per texel.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

#pragma clang fp contract(off)

namespace nsm {
namespace {

constexpr uint32_t kEmptyDepth = 0x7F800000u;
constexpr unsigned long long kEmptyKey = ~0ull;
constexpr int kScanThreads = 1024;
constexpr int kSetupThreads = 64;     // one wave per setup block: more waves in flight per CU
// Tile item shape: one texel per lane.  16 x 4 rather than 8 x 8: a wave's
// atomicMin then touches 4 rows of 64 or 128 bytes (4 cache lines) instead of
// 8, for about 9% more live items at 1080p; the atomics bound the kernel.
constexpr int kTileW = 16, kTileH = 4;
static_assert(kTileW * kTileH == 64, "one texel per lane of a wave");
constexpr int kGroup = 32;            // virtual triangles per group of the item -> triangle search
static_assert(kSetupThreads % kGroup == 0, "a search group must lie inside one setup block");
// Items are dealt to the waves in runs of kRun consecutive items, run r to
// wave r mod (waves in the grid): a wave's 64 items then sample the whole item
// list.  Consecutive items belong to one triangle and its neighbouring tiles,
// and whole runs of them cover nothing (a big triangle's bounding box around
// its diagonal), so dealing them in large contiguous chunks left some SIMDs
// with far more covered items to walk than others.
constexpr int kRun = 4;
static_assert(64 % kRun == 0, "a wave's 64 items are whole runs");
constexpr int kStep = 2;              // tile items evaluated together in the walk

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

// Clear up to two targets with 16-byte stores (a 4-byte tail loop covers
// sizes that are not multiples of 16 bytes).
struct FillJob {
    void* p;
    size_t bytes;
    unsigned long long pattern;   // 8-byte pattern repeated
};

__device__ __forceinline__ void fill2(FillJob a, FillJob b, size_t tid, size_t stride) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const FillJob f = j ? b : a;
        if (!f.p) continue;
        const size_t n16 = f.bytes / 16;
        uint4 v;
        v.x = v.z = (uint32_t)(f.pattern & 0xFFFFFFFFull);
        v.y = v.w = (uint32_t)(f.pattern >> 32);
        uint4* q = reinterpret_cast<uint4*>(f.p);
        for (size_t i = tid; i < n16; i += stride) q[i] = v;
        // tail (fewer than 16 bytes, 4-byte aligned)
        uint32_t* t32 = reinterpret_cast<uint32_t*>(f.p);
        for (size_t i = n16 * 4 + tid; i < f.bytes / 4; i += stride)
            t32[i] = (i & 1) ? (uint32_t)(f.pattern >> 32) : (uint32_t)(f.pattern & 0xFFFFFFFFull);
    }
}

// Per-triangle coefficients of the coverage and depth arithmetic, staged in
// LDS by the raster loop.  Edge k (opposite vertex k, from vertex a to vertex
// b) is E_k(px, py) = dx_k py - dy_k px + c_k with dx_k = Xb - Xa,
// dy_k = Yb - Ya, c_k = dy_k Xa - dx_k Ya: all exact integers.  104 bytes,
// so that the LDS slots of 64 records per wave allow 6 waves per SIMD.
struct alignas(8) TriCoef {
    double dx[3], dy[3], c[3];
    double area;          // doubled area (> 0)
    double inv_area;      // 1 / area rounded to nearest
    float z[3];           // vertex ndc depths
    int32_t incl;         // bit k: edge k owns the pixels exactly on it
};
static_assert(sizeof(TriCoef) == 104, "TriCoef must stay 104 bytes");

__device__ __forceinline__ bool edge_owns(int64_t dx, int64_t dy) {
    return dy > 0 || (dy == 0 && dx < 0);
}

// Snap one triangle, order it counter-clockwise and count the tiles of
// its texel bounding box (0 if dropped, degenerate or off-screen).
__device__ __forceinline__ int tri_setup_one(const float* __restrict__ tris, int t, const Mat4& M,
                                             int w, int h, TriSetup* __restrict__ setup,
                                             TriCoef* __restrict__ coef) {
    const float* T = tris + 9 * (size_t)t;
    const float fw = (float)w, fh = (float)h;
    int64_t X[3], Y[3];
    float Z[3];
    // the three vertices are transformed without early exits so that their
    // independent divisions overlap; a dropped triangle's values are unused
    bool drop = false;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        float c[4];
        to_clip(M, T[3 * v], T[3 * v + 1], T[3 * v + 2], c);
        const bool front = c[3] > 1e-6f;
        const float w = front ? c[3] : 1.0f;
        float nx = c[0] / w;
        float ny = c[1] / w;
        float nz = c[2] / w;
        float sx = (nx * 0.5f + 0.5f) * fw;
        float sy = (ny * 0.5f + 0.5f) * fh;
        const bool inside = sx >= -8.0f * fw && sx <= 9.0f * fw && sy >= -8.0f * fh && sy <= 9.0f * fh;
        drop = drop || !front || !inside;
        X[v] = inside ? (int64_t)rintf(sx * 256.0f) : 0;
        Y[v] = inside ? (int64_t)rintf(sy * 256.0f) : 0;
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
                int tx0 = (int)(i0 / kTileW), tx1 = (int)(i1 / kTileW);
                int ty0 = (int)(j0 / kTileH), ty1 = (int)(j1 / kTileH);
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
    TriCoef c;
    c.incl = 0;
    for (int k = 0; k < 3; ++k) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        const int64_t dx = (int64_t)s.x[b] - s.x[a], dy = (int64_t)s.y[b] - s.y[a];
        c.dx[k] = (double)dx;
        c.dy[k] = (double)dy;
        c.c[k] = fma((double)dy, (double)s.x[a], -((double)dx * (double)s.y[a]));
        c.z[k] = s.z[k];
        if (edge_owns(dx, dy)) c.incl |= 1 << k;
    }
    c.area = (double)s.area;
    c.inv_area = count ? 1.0 / c.area : 0.0;
    coef[t] = c;
    return count;
}

// Exclusive scan of one int per lane of a one-wave block; returns the lane's
// offset and writes the wave total to *total (all lanes call it).
__device__ __forceinline__ int wave_exclusive_scan(int v, int* total) {
    const int lane = threadIdx.x & 63;
    int incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(incl, d);
        if (lane >= d) incl += u;
    }
    *total = __shfl(incl, 63);
    return incl - v;
}

// Blocks [0, nblk) set up one virtual triangle per thread (v = pass * n_tris
// + t) and scan their tile counts; the remaining blocks clear the targets.
// The raster kernel that follows on the stream sees both finished.
__global__ void __launch_bounds__(kSetupThreads) k_tri_setup(const float* __restrict__ tris, int n_tris,
                                                   RasterPasses P, TriSetup* __restrict__ setup,
                                                   TriCoef* __restrict__ coef,
                                                   int* __restrict__ local_off, int* __restrict__ block_sum,
                                                   int nblk, FillJob fa, FillJob fb) {
    if ((int)blockIdx.x >= nblk) {
        const size_t fill_threads = (size_t)(gridDim.x - nblk) * blockDim.x;
        fill2(fa, fb, (size_t)(blockIdx.x - nblk) * blockDim.x + threadIdx.x, fill_threads);
        return;
    }
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    int count = 0;
    if (v < P.npass * n_tris) {
        const int pass = v >= n_tris ? 1 : 0;
        const RasterPass& rp = pass ? P.p[1] : P.p[0];
        count = tri_setup_one(tris, v - pass * n_tris, rp.m, rp.w, rp.h, setup + pass * n_tris,
                              coef + pass * n_tris);
    }
    int total;
    const int off = wave_exclusive_scan(count, &total);
    if (v < P.npass * n_tris) local_off[v] = off;
    if (threadIdx.x == 0) block_sum[blockIdx.x] = total;
}

// Scan of the per-block tile totals written by k_tri_setup into the start of
// every group of kGroup virtual triangles (gbase[g], gbase[ngroups] = all
// items); one block, wave-level scans.  A setup block holds two groups: the
// first starts at the block's base (its local offset is 0), the second at the
// base plus the local offset of its first triangle, which is loaded together
// with the block total, so the scan waits on one round of loads.
__global__ void __launch_bounds__(kScanThreads) k_block_scan(const int* __restrict__ block_sum, int nblk,
                                                             const int* __restrict__ local_off, int nv,
                                                             long long* __restrict__ gbase) {
    static_assert(kSetupThreads == 2 * kGroup, "two search groups per setup block");
    __shared__ long long wsum[kScanThreads / 64];
    __shared__ long long carry;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ngroups = (nv + kGroup - 1) / kGroup;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int seg = 0; seg < nblk; seg += kScanThreads) {
        const int i = seg + tid;
        const int t1 = i * kSetupThreads + kGroup;     // first triangle of block i's second group
        const long long v = (i < nblk) ? block_sum[i] : 0;
        const int lo1 = (i < nblk && t1 < nv) ? local_off[t1] : 0;
        long long incl = v;
        for (int d = 1; d < 64; d <<= 1) {
            const long long u = __shfl_up(incl, d);
            if (lane >= d) incl += u;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        long long woff = carry;
        for (int k = 0; k < wave; ++k) woff += wsum[k];
        if (i < nblk) {
            const long long b = woff + incl - v;
            gbase[2 * i] = b;
            if (2 * i + 1 < ngroups) gbase[2 * i + 1] = b + lo1;
        }
        __syncthreads();
        if (tid == kScanThreads - 1) carry = woff + incl;
        __syncthreads();
    }
    if (tid == 0) gbase[ngroups] = carry;
}

// The virtual triangle holding tile item `item` (the largest v with
// start(v) <= item) and the item's index within that triangle.  A binary
// search over the group starts (a few KB, cache resident) finds the group of
// kGroup triangles; one batch of vector loads brings the group's local
// offsets, and a branch-free pass over them finds the triangle.
__device__ __forceinline__ int find_tri(const long long* __restrict__ gbase, const int* __restrict__ local_off,
                                       int nv, long long item, int* local) {
    const int ngroups = (nv + kGroup - 1) / kGroup;
    int lo = 0, hi = ngroups;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gbase[mid] <= item) lo = mid; else hi = mid;
    }
    const int t0 = lo * kGroup;
    const int rel = (int)(item - gbase[lo]);
    const int e = min(kGroup, nv - t0);
    const int4* q = reinterpret_cast<const int4*>(local_off + t0);
    int off[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup / 4; ++u) {
        const int4 v = q[u];
        off[4 * u] = v.x; off[4 * u + 1] = v.y; off[4 * u + 2] = v.z; off[4 * u + 3] = v.w;
    }
    // offsets are non-decreasing within the group (a block-local scan), so
    // the entries <= rel form a prefix; entries past the group end are ignored
    int cnt = 0, best = 0;
#pragma unroll
    for (int i = 1; i < kGroup; ++i) {
        const int d = off[i] - off[0];
        const bool le = (i < e) & (d <= rel);
        cnt += le ? 1 : 0;
        best = le ? d : best;
    }
    *local = rel - best;
    return t0 + cnt;
}

__device__ __forceinline__ int bcast(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// False when every texel centre of tile (tx, ty) fails one edge's coverage
// test: E_k is largest at one corner of the tile's texel-centre box (the
// corner chosen by the signs of dx_k and -dy_k), and E_k <= t_k there means
// E_k > t_k holds on none of the 64 texels, so the item covers nothing.  The
// corner is a texel centre within 15 texels of the target (below 2^23 in
// 24.8 fixed point), so E_k is exact there as in the walk.
__device__ __forceinline__ bool tile_live(const TriCoef& c, int tx, int ty) {
    const double xa = (double)(256 * (kTileW * tx) + 128), xb = xa + (double)(256 * (kTileW - 1));
    const double ya = (double)(256 * (kTileH * ty) + 128), yb = ya + (double)(256 * (kTileH - 1));
    bool live = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double px = (c.dy[k] <= 0.0) ? xb : xa;
        const double py = (c.dx[k] >= 0.0) ? yb : ya;
        const double e = fma(c.dx[k], py, fma(-c.dy[k], px, c.c[k]));
        live = live && (e > (((c.incl >> k) & 1) ? -1.0 : 0.0));
    }
    return live;
}

// One (triangle, tile) item, one texel per lane: the texel's depth
// candidate, evaluated without branches so that the walk can interleave the
// dependent float64 chains of two items.  `ok` is false where the texel is
// outside the target, not covered, or outside the depth range.
struct Frag {
    bool ok, pass;
    uint32_t bits, t;
    int i, j, rw;
};

__device__ __forceinline__ Frag raster_eval(const TriCoef& c, int vk, int tx, int ty, int lx, int ly, int n_tris,
                                            int w0, int h0, int w1, int h1) {
    Frag f;
    f.pass = vk >= n_tris;
    f.t = (uint32_t)(vk - (f.pass ? n_tris : 0));
    f.rw = f.pass ? w1 : w0;
    const int rh = f.pass ? h1 : h0;
    f.i = tx * kTileW + lx;
    f.j = ty * kTileH + ly;
    const double px = (double)(256 * f.i + 128), py = (double)(256 * f.j + 128);
    const double e0 = fma(c.dx[0], py, fma(-c.dy[0], px, c.c[0]));
    const double e1 = fma(c.dx[1], py, fma(-c.dy[1], px, c.c[1]));
    const double e2 = fma(c.dx[2], py, fma(-c.dy[2], px, c.c[2]));
    // E_k is an integer, so the tie rule "E > 0, or E == 0 on an owned edge"
    // is E > t_k with t_k = -1 on owned edges and 0 otherwise; the record is
    // the same for the whole wave, so the thresholds live in scalar registers
    const int incl = __builtin_amdgcn_readfirstlane(c.incl);
    const double t0 = (incl & 1) ? -1.0 : 0.0, t1 = (incl & 2) ? -1.0 : 0.0, t2 = (incl & 4) ? -1.0 : 0.0;
    const bool cov = (e0 > t0) & (e1 > t1) & (e2 > t2) & (f.i < f.rw) & (f.j < rh);
    double num = e0 * (double)c.z[0];
    num = num + e1 * (double)c.z[1];
    num = num + e2 * (double)c.z[2];
    const double q0 = num * c.inv_area;
    const double q = fma(fma(-q0, c.area, num), c.inv_area, q0);
    const float d = (float)q;
    f.ok = cov & (d >= 0.0f) & (d <= 1.0f);
    uint32_t bits = __float_as_uint(d);
    if ((bits & 0x7FFFFFFFu) == 0) bits = 0;  // -0 -> +0
    f.bits = bits;
    return f;
}

__device__ __forceinline__ void raster_store(const Frag& f, bool k0, bool k1, void* o0, void* o1) {
    if (!f.ok) return;
    const size_t o = (size_t)f.j * (size_t)f.rw + (size_t)f.i;
    if (f.pass ? k1 : k0) {
        const unsigned long long key = ((unsigned long long)f.bits << 32) | (unsigned long long)f.t;
        atomicMin(reinterpret_cast<unsigned long long*>(f.pass ? o1 : o0) + o, key);
    } else {
        atomicMin(reinterpret_cast<uint32_t*>(f.pass ? o1 : o0) + o, f.bits);
    }
}

// Each wave takes 64 tile items at a time (16 runs of kRun consecutive items,
// strided over the item list; the grid is the number of blocks the device
// holds at once).  Lane k first finds the triangle and tile of its item (64
// searches in flight at once), stages that triangle's coefficient record in
// LDS and tests whether the tile can hold a covered texel (about 40% of
// bounding-box tiles cannot); the wave then walks the live items, one lane per
// texel of the tile.
// Inside the walk nothing waits on vector memory: the depth update is a
// fire-and-forget integer atomicMin.
//
// All coverage arithmetic is float64 on exact integers: snapped coordinates
// lie in the guard band [-8 S, 9 S] (S <= 16384 texels, 8 subpixel bits), so
// |X| < 2^25.2, edge deltas are below 2^26.1, |c_k| < 2^52.3 and, with texel
// centres (and the culling test's tile corners) below 2^23, every product and
// partial sum of E_k is an integer under 2^53: each E_k is exact (what 64-bit
// integer arithmetic gives).  The depth
// quotient num / area is rounded correctly with one fused correction of
// num * (1 / area) (Markstein's theorem: the reciprocal is rounded to nearest
// and the first quotient is within one ulp), so it equals the IEEE division.
__global__ void __launch_bounds__(256) k_raster(const TriSetup* __restrict__ setup,
                                                const TriCoef* __restrict__ coef,
                                                const long long* __restrict__ gbase,
                                                const int* __restrict__ local_off, int n_tris,
                                                RasterPasses P) {
    const int lane = threadIdx.x & 63;
    const int nv = P.npass * n_tris;             // virtual triangles
    const long long total = gbase[(nv + kGroup - 1) / kGroup];
    const long long nwaves = (long long)gridDim.x * (blockDim.x >> 6);
    const int w0 = P.p[0].w, h0 = P.p[0].h, w1 = P.p[1].w, h1 = P.p[1].h;
    const bool k0 = P.p[0].key64, k1 = P.p[1].key64;
    void* const o0 = P.p[0].out;
    void* const o1 = P.p[1].out;
    const int lx = lane % kTileW, ly = lane / kTileW;
    __shared__ TriCoef lcoef[4][64];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long wid = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    // round q0 of this wave: lane k takes item kRun * (((q0 + k) / kRun) * nwaves + wid) + (q0 + k) % kRun
    for (long long q0 = 0; (q0 / kRun * nwaves + wid) * kRun < total; q0 += 64) {
        const long long q = q0 + lane;
        const long long item = (q / kRun * nwaves + wid) * kRun + q % kRun;
        int v = 0, tx = 0, ty = 0;
        bool live = false;
        if (item < total) {
            int local;
            v = find_tri(gbase, local_off, nv, item, &local);
            const int ntx = setup[v].ntx;
            tx = setup[v].tx0 + local % ntx;
            ty = setup[v].ty0 + local / ntx;
        }
        // lane k stages its item's coefficient record in the wave's LDS slots
        // (64 vector loads in flight at once) and tests whether the tile can
        // hold a covered texel at all; the walk then reads each live item's
        // record with same-address (broadcast) LDS reads
        {
            TriCoef cl;
            const uint2* src = reinterpret_cast<const uint2*>(coef + v);
            uint2* tmp = reinterpret_cast<uint2*>(&cl);
            uint2* dst = reinterpret_cast<uint2*>(&lcoef[wv][lane]);
#pragma unroll
            for (int u = 0; u < (int)(sizeof(TriCoef) / 8); ++u) {
                tmp[u] = src[u];
                dst[u] = tmp[u];
            }
            live = item < total && tile_live(cl, tx, ty);
        }
        // the round's live items, in order (a wave-uniform lane mask)
        unsigned long long todo = __ballot(live);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // kStep live items per step: their records are read together and
        // their independent float64 chains are all evaluated before the first
        // store, so the chains overlap; past the last live item a step repeats
        // its first item (a repeated atomicMin changes nothing)
        while (todo) {
            int ks[kStep];
            ks[0] = __builtin_ctzll(todo);
            todo &= todo - 1;
#pragma unroll
            for (int u = 1; u < kStep; ++u) {
                ks[u] = todo ? __builtin_ctzll(todo) : ks[0];
                todo &= todo - 1;
            }
            TriCoef cr[kStep];
#pragma unroll
            for (int u = 0; u < kStep; ++u) cr[u] = lcoef[wv][ks[u]];
            Frag fr[kStep];
#pragma unroll
            for (int u = 0; u < kStep; ++u) {
                const int ku = ks[u];
                fr[u] = raster_eval(cr[u], bcast(v, ku), bcast(tx, ku), bcast(ty, ku), lx, ly, n_tris, w0, h0, w1,
                                    h1);
            }
            // keep the evaluations above the stores (the compiler would otherwise
            // sink each chain below the previous item's store branch)
#pragma unroll
            for (int u = 0; u < kStep; ++u) asm volatile("" ::"v"(fr[u].bits), "v"((int)fr[u].ok));
#pragma unroll
            for (int u = 0; u < kStep; ++u) raster_store(fr[u], k0, k1, o0, o1);
        }
        // the slots are rewritten for the next round only after every lane is done reading
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__device__ __forceinline__ float lin_depth(float q, float nl, float fl) {
    float num = nl * fl;
    float den = fl - q * (fl - nl);
    return num / den;
}

// Linear light-view depth of every shadow-map texel, +inf where the map is
// empty: the SOFT8 blocker search reads 49 texels per pixel, and this turns
// their 49 divisions into one per texel.  lin_depth is a pure function of the
// texel, so the search sees the same values either way.  Four texels per
// thread (16-byte accesses); the tail runs one per thread.
__global__ void __launch_bounds__(256) k_linear_map(const uint32_t* __restrict__ sm, size_t n, float nl, float fl,
                                                    float* __restrict__ lsm) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n4 = n / 4;
    if (i < n4) {
        const uint4 b = reinterpret_cast<const uint4*>(sm)[i];
        float4 o;
        o.x = b.x == kEmptyDepth ? __uint_as_float(kEmptyDepth) : lin_depth(__uint_as_float(b.x), nl, fl);
        o.y = b.y == kEmptyDepth ? __uint_as_float(kEmptyDepth) : lin_depth(__uint_as_float(b.y), nl, fl);
        o.z = b.z == kEmptyDepth ? __uint_as_float(kEmptyDepth) : lin_depth(__uint_as_float(b.z), nl, fl);
        o.w = b.w == kEmptyDepth ? __uint_as_float(kEmptyDepth) : lin_depth(__uint_as_float(b.w), nl, fl);
        reinterpret_cast<float4*>(lsm)[i] = o;
    } else if (i < n4 + (n & 3)) {
        const size_t t = 4 * n4 + (i - n4);
        const uint32_t b = sm[t];
        lsm[t] = b == kEmptyDepth ? __uint_as_float(kEmptyDepth) : lin_depth(__uint_as_float(b), nl, fl);
    }
}

// FS: 0 = HARD6, 1 = SOFT8, 2 = PAPER4
//
// Each thread carries kGatherPx pixels of one row (stride 256) through the
// three dependent fetches -- camera key, then the key's triangle, then the
// shadow-map texel -- one stage at a time, all loads unconditional (triangle
// 0 and texel 0 stand in where a pixel has none).  Measured on the 1080p
// frame, one pixel per thread with more waves in flight beats four per
// thread: the gather is bound by its vector ALU work as much as by latency.
constexpr int kGatherPx = 1;
constexpr int kWinCap = 1024;     // texels of a wave's staged window box (4 KB of LDS)

// OD selects how the channels are written: 0 float32 [h][w][C]; 1 bfloat16
// and 2 float16 [h][w][8], each float32 channel rounded to nearest even and
// the channels past C zero (the network's storage type, read by its first
// stage as whole 16-byte blocks); 3 FP8 E4M3 bytes [h][w][16], each channel
// saturated to +-448 and rounded to nearest even by the hardware
// conversion, the bytes past C zero.
template <int FS, int OD>
__global__ void __launch_bounds__(256) k_gather(const float* __restrict__ tris,
                                                const float* __restrict__ normals, int n_tris,
                                                GatherParams P,
                                                const unsigned long long* __restrict__ gbuf,
                                                const uint32_t* __restrict__ sm, const float* __restrict__ lsm,
                                                int w, int h, void* __restrict__ feat,
                                                uint8_t* __restrict__ mask) {
    constexpr bool SOFT = FS == 1;
    constexpr int C = FS == 1 ? 8 : (FS == 2 ? 4 : 6);
    constexpr int PX = kGatherPx;
    // 16 x 16 pixels per block, 8 x 8 per wave: compact shadow-map footprints
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int j = blockIdx.y * 16 + (wv >> 1) * 8 + (ln >> 3);
    const int ib = blockIdx.x * 16 + (wv & 1) * 8 + (ln & 7);
    // stage 1: camera keys
    unsigned long long key[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int i = ib + 256 * k;
        key[k] = (i < w && j < h) ? gbuf[(size_t)j * (size_t)w + (size_t)i] : kEmptyKey;
    }
    // stage 2: the keys' triangles (vertex 0 and the face normal)
    float V0[PX][3], N[PX][3];
    bool fg[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const uint32_t t = (uint32_t)(key[k] & 0xFFFFFFFFull);
        fg[k] = key[k] != kEmptyKey && (int)t < n_tris;
        const size_t tc = fg[k] ? t : 0;          // triangle 0 stands in for background pixels
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            V0[k][d] = n_tris > 0 ? tris[9 * tc + d] : 0.0f;
            N[k][d] = n_tris > 0 ? normals[3 * tc + d] : 0.0f;
        }
    }
    // stage 3: receiver, light-view projection, texel address
    double D[PX][3], tt[PX];
    float Pw[PX][3], c3[PX][4];
    bool inside[PX];
    float zf[PX];
    int ti[PX], tj[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int i = ib + 256 * k;
        tt[k] = 0.0;
        // receiver: the pixel-centre camera ray meets the triangle's plane
        // (float64).  The quotients (2 i + 1) / w and (2 j + 1) / h are the
        // correctly rounded ones, from the rounded reciprocal and one
        // Markstein correction (Markstein's theorem; the operands are positive
        // integers below 2^15, and every pair up to 16384 was checked against
        // the IEEE division).
        const double ax2 = 2.0 * ((double)i + 0.5), ay2 = 2.0 * ((double)j + 0.5);
        const double qx0 = ax2 * P.rw, qy0 = ay2 * P.rh;
        const double ndcx = fma(fma(-qx0, (double)w, ax2), P.rw, qx0) - 1.0;
        const double ndcy = fma(fma(-qy0, (double)h, ay2), P.rh, qy0) - 1.0;
        const double ax = ndcx * P.tanx_d, ay = ndcy * P.tany_d;
#pragma unroll
        for (int d = 0; d < 3; ++d) D[k][d] = (P.fwd_d[d] + ax * P.right_d[d]) + ay * P.up_d[d];
        double num = (double)N[k][0] * ((double)V0[k][0] - P.E_d[0]);
        num = num + (double)N[k][1] * ((double)V0[k][1] - P.E_d[1]);
        num = num + (double)N[k][2] * ((double)V0[k][2] - P.E_d[2]);
        double den = (double)N[k][0] * D[k][0];
        den = den + (double)N[k][1] * D[k][1];
        den = den + (double)N[k][2] * D[k][2];
        if (den == 0.0) fg[k] = false;
        else tt[k] = num / den;
#pragma unroll
        for (int d = 0; d < 3; ++d) Pw[k][d] = (float)(P.E_d[d] + tt[k] * D[k][d]);
        to_clip(P.ml, Pw[k][0], Pw[k][1], Pw[k][2], c3[k]);
        inside[k] = fg[k] && c3[k][3] > 1e-6f;
        zf[k] = P.fl;
        ti[k] = 0;
        tj[k] = 0;
        if (inside[k]) {
            const float nx = c3[k][0] / c3[k][3], ny = c3[k][1] / c3[k][3], nz = c3[k][2] / c3[k][3];
            const float sx = (nx * 0.5f + 0.5f) * (float)P.S;
            const float sy = (ny * 0.5f + 0.5f) * (float)P.S;
            zf[k] = lin_depth(nz, P.nl, P.fl);
            inside[k] = sx >= 0.0f && sx < (float)P.S && sy >= 0.0f && sy < (float)P.S && nz >= 0.0f &&
                        nz <= 1.0f;
            if (inside[k]) {
                ti[k] = (int)floorf(sx);
                tj[k] = (int)floorf(sy);
            }
        }
    }
    // stage 4: shadow-map texels
    uint32_t tex[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) tex[k] = sm[(size_t)tj[k] * (size_t)P.S + (size_t)ti[k]];
    // stage 4b (SOFT8): when the 7x7 windows of the wave's 8 x 8 pixels fit a
    // small box of the map, the wave stages that box in LDS (one coalesced
    // row per load) and the blocker search reads it from there
    bool win_lds = false, win_full = false;
    int wx0 = 0, wy0 = 0, wrw = 1;
    __shared__ float win[4][kWinCap];
    if constexpr (SOFT) {
        static_assert(PX == 1, "the window box assumes one pixel per lane");
        const bool part = inside[0];
        int imin = part ? ti[0] : 0x7FFFFFFF, imax = part ? ti[0] : -1;
        int jmin = part ? tj[0] : 0x7FFFFFFF, jmax = part ? tj[0] : -1;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            imin = min(imin, __shfl_xor(imin, d));
            imax = max(imax, __shfl_xor(imax, d));
            jmin = min(jmin, __shfl_xor(jmin, d));
            jmax = max(jmax, __shfl_xor(jmax, d));
        }
        // the same in every lane after the butterfly: scalar from here on
        imin = __builtin_amdgcn_readfirstlane(imin);
        imax = __builtin_amdgcn_readfirstlane(imax);
        jmin = __builtin_amdgcn_readfirstlane(jmin);
        jmax = __builtin_amdgcn_readfirstlane(jmax);
        if (imax >= 0) {
            wx0 = max(imin - 3, 0);
            wy0 = max(jmin - 3, 0);
            wrw = min(imax + 3, P.S - 1) - wx0 + 1;
            const int rh = min(jmax + 3, P.S - 1) - wy0 + 1;
            win_lds = wrw <= 64 && wrw * rh <= kWinCap;
            // no window of the wave reaches past the map: every tap is in the
            // box, unclamped and unmasked
            win_full = win_lds && imin >= 3 && jmin >= 3 && imax + 3 <= P.S - 1 && jmax + 3 <= P.S - 1;
            if (win_lds) {
                for (int r = 0; r < rh; ++r)
                    if (ln < wrw) win[wv][r * wrw + ln] = lsm[(size_t)(wy0 + r) * (size_t)P.S + (size_t)(wx0 + ln)];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
    // stage 5: features and mask
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int i = ib + 256 * k;
        if (i >= w || j >= h) continue;
        const size_t p = (size_t)j * (size_t)w + (size_t)i;
        float f[C];
#pragma unroll
        for (int c = 0; c < C; ++c) f[c] = 0.0f;
        uint8_t mk = 0;
        if (fg[k]) {
            float n0 = N[k][0], n1 = N[k][1], n2 = N[k][2];
            const float vx = P.E[0] - Pw[k][0], vy = P.E[1] - Pw[k][1], vz = P.E[2] - Pw[k][2];
            float sgn = n0 * vx + n1 * vy;
            sgn = sgn + n2 * vz;
            if (sgn < 0.0f) { n0 = -n0; n1 = -n1; n2 = -n2; }
            float dv = (Pw[k][0] - P.E[0]) * P.fwd[0] + (Pw[k][1] - P.E[1]) * P.fwd[1];
            dv = dv + (Pw[k][2] - P.E[2]) * P.fwd[2];
            bool ins = inside[k];
            float z = P.fl;
            if (ins) {
                if (tex[k] == kEmptyDepth) ins = false;
                else z = lin_depth(__uint_as_float(tex[k]), P.nl, P.fl);
            }
            // slope-scaled depth bias from the angle between normal and light direction
            const float tau = P.tau;
            const float lx = P.L[0] - Pw[k][0], ly = P.L[1] - Pw[k][1], lz = P.L[2] - Pw[k][2];
            float ll = lx * lx + ly * ly;
            ll = ll + lz * lz;
            const float len = sqrtf(ll);
            const float hx = lx / len, hy = ly / len, hz = lz / len;
            float cl = n0 * hx + n1 * hy;
            cl = cl + n2 * hz;
            const float sn = sqrtf(fmaxf(1.0f - cl * cl, 0.0f));
            const float tq = sn / fmaxf(cl, 1e-3f);
            const float beta = (zf[k] * tau) * (1.0f + 1.5f * fminf(tq, 10.0f));
            mk = (ins && zf[k] > z + beta) ? 1 : 0;
            if constexpr (FS == 2) {
                // c_e with the emitter-size offset, z/z_f, z - z_f, c_c/d
                float vv = vx * vx + vy * vy;
                vv = vv + vz * vz;
                float cc = n0 * vx + n1 * vy;
                cc = cc + n2 * vz;
                cc = cc / sqrtf(vv);
                f[0] = cl + P.r_e / 0.0625f;
                f[1] = z / zf[k];
                f[2] = (z - zf[k]) / P.fl;
                f[3] = cc / dv;
            } else {
                f[0] = dv / P.fc;
                f[1] = n0;
                f[2] = n1;
                f[3] = n2;
                f[4] = (z - zf[k]) / P.fl;
                f[5] = z / P.fl;
            }
            if constexpr (SOFT) {
                float zb = zf[k];
                if (ins) {
                    const float thr = zf[k] - beta;
                    float sum = 0.0f;
                    int cnt = 0;
                    if (win_full) {
                        // tap (dj, di) is box element (tj + dj - wy0, ti + di - wx0)
                        const float* wb = &win[wv][(tj[k] - 3 - wy0) * wrw + (ti[k] - 3 - wx0)];
                        float qv[49];
#pragma unroll
                        for (int dj = 0; dj < 7; ++dj)
#pragma unroll
                            for (int di = 0; di < 7; ++di) qv[dj * 7 + di] = wb[dj * wrw + di];
#pragma unroll
                        for (int t = 0; t < 49; ++t)
                            if (qv[t] < thr) { sum = sum + qv[t]; ++cnt; }
                    } else {
                        // all 49 loads issued together: indices clamped into the map,
                        // out-of-map taps masked (the same taps, summed in the same order)
                        float qv[49];
#pragma unroll
                        for (int dj = -3; dj <= 3; ++dj) {
                            const int jj = min(max(tj[k] + dj, 0), P.S - 1);
#pragma unroll
                            for (int di = -3; di <= 3; ++di) {
                                const int ii = min(max(ti[k] + di, 0), P.S - 1);
                                qv[(dj + 3) * 7 + di + 3] = win_lds ? win[wv][(jj - wy0) * wrw + (ii - wx0)]
                                                                    : lsm[(size_t)jj * (size_t)P.S + (size_t)ii];
                            }
                        }
#pragma unroll
                        for (int dj = -3; dj <= 3; ++dj) {
                            const bool okj = tj[k] + dj >= 0 && tj[k] + dj < P.S;
#pragma unroll
                            for (int di = -3; di <= 3; ++di) {
                                const bool ok = okj && ti[k] + di >= 0 && ti[k] + di < P.S;
                                // +inf where the map is empty: never below the threshold
                                const float q = qv[(dj + 3) * 7 + di + 3];
                                if (ok && q < thr) { sum = sum + q; ++cnt; }
                            }
                        }
                    }
                    if (cnt > 0) zb = sum / (float)cnt;
                }
                f[C - 2] = P.r_e / 0.2f;
                f[C - 1] = zb / P.fl;
            }
        }
        if constexpr (OD == 0) {
            float* o = reinterpret_cast<float*>(feat) + p * C;
#pragma unroll
            for (int c = 0; c < C; ++c) o[c] = f[c];
        } else if constexpr (OD == 3) {
            static_assert(C <= 8, "one 16-byte block per pixel");
            float c8[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) c8[c] = c < C ? __builtin_amdgcn_fmed3f(f[c], 448.0f, -448.0f) : 0.0f;
            uint4 v;
            int lo = __builtin_amdgcn_cvt_pk_fp8_f32(c8[0], c8[1], 0, false);
            lo = __builtin_amdgcn_cvt_pk_fp8_f32(c8[2], c8[3], lo, true);
            int hi = __builtin_amdgcn_cvt_pk_fp8_f32(c8[4], c8[5], 0, false);
            hi = __builtin_amdgcn_cvt_pk_fp8_f32(c8[6], c8[7], hi, true);
            v.x = (unsigned)lo;
            v.y = (unsigned)hi;
            v.z = 0u;
            v.w = 0u;
            reinterpret_cast<uint4*>(feat)[p] = v;
        } else {
            static_assert(C <= 8, "one 16-byte block per pixel");
            using T = typename std::conditional<OD == 1, __bf16, _Float16>::type;
            typedef T t8 __attribute__((ext_vector_type(8)));
            t8 v;
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = c < C ? (T)f[c] : (T)0.0f;
            reinterpret_cast<t8*>(feat)[p] = v;
        }
        if (mask) mask[p] = mk;
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t raster_workspace_bytes(int n_tris) {
    const size_t nv = 2 * (size_t)n_tris, nblk = (nv + kSetupThreads - 1) / kSetupThreads,
                 ng = (nv + kGroup - 1) / kGroup;
    return align256(nv * sizeof(TriSetup)) + align256(nv * sizeof(TriCoef)) + align256(nv * 4) +
           align256(nblk * 4) + align256((ng + 1) * 8);
}

hipError_t raster(const float* tris, int n_tris, const RasterPasses& P, void* ws, hipStream_t s) {
    const char* sfx = P.npass == 2 ? " light+camera" : (P.p[0].key64 ? " camera" : " light");
    FillJob f[2] = {{nullptr, 0, 0}, {nullptr, 0, 0}};
    size_t most = 0;
    for (int k = 0; k < P.npass; ++k) {
        const RasterPass& rp = P.p[k];
        f[k].p = rp.out;
        f[k].bytes = (size_t)rp.w * rp.h * (rp.key64 ? 8 : 4);
        f[k].pattern = rp.key64 ? kEmptyKey : (((unsigned long long)kEmptyDepth << 32) | kEmptyDepth);
        most = max(most, f[k].bytes);
    }
    const int nv = P.npass * n_tris;
    const int nblk = (nv + kSetupThreads - 1) / kSetupThreads;
    char* wsb = reinterpret_cast<char*>(ws);
    TriSetup* setup = reinterpret_cast<TriSetup*>(wsb);
    wsb += align256((size_t)nv * sizeof(TriSetup));
    TriCoef* coef = reinterpret_cast<TriCoef*>(wsb);
    wsb += align256((size_t)nv * sizeof(TriCoef));
    int* local_off = reinterpret_cast<int*>(wsb);
    wsb += align256((size_t)nv * 4);
    int* block_sum = reinterpret_cast<int*>(wsb);
    wsb += align256((size_t)nblk * 4);
    long long* gbase = reinterpret_cast<long long*>(wsb);
    {
        TraceScope ts("setup+clear", sfx, s);
        const int fill_blocks = (int)min((size_t)4096, (most / 16 + kSetupThreads - 1) / kSetupThreads + 1);
        k_tri_setup<<<nblk + fill_blocks, kSetupThreads, 0, s>>>(tris, n_tris, P, setup, coef, local_off, block_sum, nblk,
                                                       f[0], f[1]);
    }
    if (n_tris == 0) return hipGetLastError();
    {
        TraceScope ts("tile_scan", sfx, s);
        k_block_scan<<<1, kScanThreads, 0, s>>>(block_sum, nblk, local_off, nv, gbase);
    }
    {
        TraceScope ts("raster", sfx, s);
        // every wave resident at once, so that the dealt items spread evenly over the SIMDs
        static const int blocks = [] {
            int dev = 0, cus = 256, per = 1;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_raster, 256, 0) != hipSuccess || per < 1) per = 1;
            return per * cus;
        }();
        k_raster<<<blocks, 256, 0, s>>>(setup, coef, gbase, local_off, n_tris, P);
    }
    return hipGetLastError();
}

size_t linear_map_bytes(int sm_size) { return align256((size_t)sm_size * (size_t)sm_size * 4); }

hipError_t gather(const float* tris, const float* normals, int n_tris, const GatherParams& params,
                  const uint64_t* gbuf, const uint32_t* sm, float* lsm, int w, int h, int fs, int od, void* feat,
                  uint8_t* mask, hipStream_t s) {
    if (od < 0 || od > 3 || (od != 0 && fs == 2)) return hipErrorInvalidValue;
    GatherParams p = params;
    p.tau = (2.0f * p.tanl) / (float)p.S;
    p.rw = 1.0 / (double)w;
    p.rh = 1.0 / (double)h;
    for (int d = 0; d < 3; ++d) {
        p.E_d[d] = (double)p.E[d];
        p.fwd_d[d] = (double)p.fwd[d];
        p.right_d[d] = (double)p.right[d];
        p.up_d[d] = (double)p.up[d];
    }
    p.tanx_d = (double)p.tanx;
    p.tany_d = (double)p.tany;
    static_assert(kGatherPx == 1, "one pixel per thread");
    dim3 grid((w + 15) / 16, (h + 15) / 16);
    const auto* g = reinterpret_cast<const unsigned long long*>(gbuf);
    if (fs == 1) {
        const size_t n = (size_t)p.S * (size_t)p.S;
        const size_t threads = n / 4 + (n & 3);
        TraceScope ts("linear_map", "", s);
        k_linear_map<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(sm, n, p.nl, p.fl, lsm);
    }
    static const char* const names[2][3] = {{" hard6", " soft8", " paper4"}, {" hard6 stored", " soft8 stored", ""}};
    TraceScope ts("gather", names[od != 0][fs], s);
    if (fs == 1) {
        if (od == 1)
            k_gather<1, 1><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, lsm, w, h, feat, mask);
        else if (od == 2)
            k_gather<1, 2><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, lsm, w, h, feat, mask);
        else if (od == 3)
            k_gather<1, 3><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, lsm, w, h, feat, mask);
        else
            k_gather<1, 0><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, lsm, w, h, feat, mask);
    } else if (fs == 2) {
        k_gather<2, 0><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, nullptr, w, h, feat, mask);
    } else {
        if (od == 1)
            k_gather<0, 1><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, nullptr, w, h, feat, mask);
        else if (od == 2)
            k_gather<0, 2><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, nullptr, w, h, feat, mask);
        else if (od == 3)
            k_gather<0, 3><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, nullptr, w, h, feat, mask);
        else
            k_gather<0, 0><<<grid, 256, 0, s>>>(tris, normals, n_tris, p, g, sm, nullptr, w, h, feat, mask);
    }
    return hipGetLastError();
}

}  // namespace nsm
