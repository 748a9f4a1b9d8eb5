// Device helpers shared by the direction-independent kernels: complex and 2x2 algebra,
// wavefront/workgroup reductions and the per-antenna GN value.
#pragma once

#include "wcal_internal.h"

namespace wcal_dev {

constexpr int WAVE = 64;

// ------------------------------------------------------------------ complex helpers
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ __forceinline__ float2 ccmul(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float nrm(float2 a) { return a.x * a.x + a.y * a.y; }

struct J2 { float2 a, b, c, d; };   // 2x2 row-major: [[a, b], [c, d]]

__device__ __forceinline__ J2 mul(const J2& x, const J2& y) {
    J2 r;
    r.a = cadd(cmul(x.a, y.a), cmul(x.b, y.c));
    r.b = cadd(cmul(x.a, y.b), cmul(x.b, y.d));
    r.c = cadd(cmul(x.c, y.a), cmul(x.d, y.c));
    r.d = cadd(cmul(x.c, y.b), cmul(x.d, y.d));
    return r;
}
// x * y^H
__device__ __forceinline__ J2 mulH(const J2& x, const J2& y) {
    J2 r;
    r.a = cadd(cmulc(x.a, y.a), cmulc(x.b, y.b));
    r.b = cadd(cmulc(x.a, y.c), cmulc(x.b, y.d));
    r.c = cadd(cmulc(x.c, y.a), cmulc(x.d, y.b));
    r.d = cadd(cmulc(x.c, y.c), cmulc(x.d, y.d));
    return r;
}
// x^H * y
__device__ __forceinline__ J2 Hmul(const J2& x, const J2& y) {
    J2 r;
    r.a = cadd(ccmul(x.a, y.a), ccmul(x.c, y.c));
    r.b = cadd(ccmul(x.a, y.b), ccmul(x.c, y.d));
    r.c = cadd(ccmul(x.b, y.a), ccmul(x.d, y.c));
    r.d = cadd(ccmul(x.b, y.b), ccmul(x.d, y.d));
    return r;
}
__device__ __forceinline__ J2 jsub(const J2& x, const J2& y) {
    return J2{csub(x.a, y.a), csub(x.b, y.b), csub(x.c, y.c), csub(x.d, y.d)};
}

__device__ __forceinline__ J2 load_j2(const float2* base, int64_t row) {
    const float4* p = reinterpret_cast<const float4*>(base) + 2 * row;
    float4 u = p[0], v = p[1];
    return J2{make_float2(u.x, u.y), make_float2(u.z, u.w), make_float2(v.x, v.y), make_float2(v.z, v.w)};
}
__device__ __forceinline__ void store_j2(float2* base, int64_t row, const J2& x) {
    float4* p = reinterpret_cast<float4*>(base) + 2 * row;
    p[0] = make_float4(x.a.x, x.a.y, x.b.x, x.b.y);
    p[1] = make_float4(x.c.x, x.c.y, x.d.x, x.d.y);
}

// ------------------------------------------------------------------ reductions
// Segmented inclusive scan across the wavefront over runs of equal `key` (lanes in
// order), then the last lane of each run adds the run total into acc[key * stride + i].
// Lanes with key < 0 contribute nothing.  Every lane of the wavefront must call this.
template <int NV>
__device__ __forceinline__ void seg_add(int key, float (&v)[NV], float* acc, int stride) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int prev = __shfl_up(key, 1, WAVE);
    int rs = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        int t = __shfl_up(rs, off, WAVE);
        if (lane >= off) rs = max(rs, t);
    }
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            float t = __shfl_up(v[i], off, WAVE);
            if (lane - off >= rs) v[i] += t;
        }
    }
    const int next = __shfl_down(key, 1, WAVE);
    const bool tail = (lane == WAVE - 1) || (next != key);
    if (tail && key >= 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) atomicAdd(&acc[key * stride + i], v[i]);
    }
}

__device__ __forceinline__ void seg_add_int(int key, int v, int* acc) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int prev = __shfl_up(key, 1, WAVE);
    int rs = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        int t = __shfl_up(rs, off, WAVE);
        if (lane >= off) rs = max(rs, t);
    }
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        int t = __shfl_up(v, off, WAVE);
        if (lane - off >= rs) v += t;
    }
    const int next = __shfl_down(key, 1, WAVE);
    const bool tail = (lane == WAVE - 1) || (next != key);
    if (tail && key >= 0) atomicAdd(&acc[key], v);
}

// element i (0 <= i, i * sizeof(T) < 2^32) of an array that starts at `base`, a
// wavefront-uniform pointer, via a 32-bit byte offset so the load takes the scalar-base form
template <typename T>
__device__ __forceinline__ T load_at(const T* base, int i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)i * (uint32_t)sizeof(T));
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

// Sum of x over the workgroup; `red` holds >= blockDim/64 doubles.  Result valid in every
// thread.  Contains barriers: call from uniform control flow only.
__device__ inline double block_sum(double x, double* red) {
    x = wave_sum(x);
    const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[w] = x;
    __syncthreads();
    double t = 0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// acc[0][i] = sum over wavefronts w (in order) of acc[w][i], i < n.  Barrier before return.
__device__ inline void fold_waves(float* acc, int n) {
    const int nw = blockDim.x / WAVE;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        float t = acc[i];
        for (int w = 1; w < nw; ++w) t += acc[w * n + i];
        acc[i] = t;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ per-row work
// Number of floats accumulated per antenna.  MODE 0 = solve (J^H J block + J^H D),
// MODE 1 = accumulate (adds J^H r).
template <int NC, int MODE> struct Nv;
template <> struct Nv<1, 0> { static constexpr int v = 3; };
template <> struct Nv<1, 1> { static constexpr int v = 5; };
template <> struct Nv<4, 0> { static constexpr int v = 12; };
template <> struct Nv<4, 1> { static constexpr int v = 20; };

__device__ __forceinline__ bool avg_step(int k, int schedule) {
    return schedule == WCAL_AVG_FIRST ? (k % 2 == 0) : schedule == WCAL_GN_FIRST ? (k % 2 == 1) : false;
}

// Per-antenna GN value in FP64.  Returns false when the block is singular (gain kept).
template <int NC>
__device__ bool gn_value(const float* ac, const float2* g, double (&gh)[2 * NC], bool& finite) {
    if constexpr (NC == 1) {
        const double A = ac[0], cr = ac[1], ci = ac[2];
        finite = isfinite(A) && isfinite(cr) && isfinite(ci);
        if (!(A > 0.0)) { gh[0] = g[0].x; gh[1] = g[0].y; return false; }
        gh[0] = cr / A; gh[1] = ci / A;
        return true;
    } else {
        bool fin = true;
#pragma unroll
        for (int i = 0; i < 12; ++i) fin = fin && isfinite(ac[i]);
        finite = fin;
        const double z00 = ac[0], z11 = ac[1], zr = ac[2], zi = ac[3];
        const double det = z00 * z11 - (zr * zr + zi * zi);
        if (!(z00 > 0.0) || !(det > WCAL_EPS_PIVOT * z00 * z11)) {
#pragma unroll
            for (int i = 0; i < 4; ++i) { gh[2 * i] = g[i].x; gh[2 * i + 1] = g[i].y; }
            return false;
        }
        const double inv = 1.0 / det;
        // Z^-1 = [[z11, -z01], [-conj(z01), z00]] / det ; G = N Z^-1
        const double nar = ac[4], nai = ac[5], nbr = ac[6], nbi = ac[7];
        const double ncr = ac[8], nci = ac[9], ndr = ac[10], ndi = ac[11];
        // row 0: [na, nb] ; row 1: [nc, nd]
        // G00 = na z11 - nb conj(z01) ; G01 = -na z01 + nb z00
        gh[0] = (nar * z11 - (nbr * zr + nbi * zi)) * inv;
        gh[1] = (nai * z11 - (nbi * zr - nbr * zi)) * inv;
        gh[2] = (-(nar * zr - nai * zi) + nbr * z00) * inv;
        gh[3] = (-(nar * zi + nai * zr) + nbi * z00) * inv;
        gh[4] = (ncr * z11 - (ndr * zr + ndi * zi)) * inv;
        gh[5] = (nci * z11 - (ndi * zr - ndr * zi)) * inv;
        gh[6] = (-(ncr * zr - nci * zi) + ndr * z00) * inv;
        gh[7] = (-(ncr * zi + nci * zr) + ndi * z00) * inv;
        return true;
    }
}

}  // namespace wcal_dev
