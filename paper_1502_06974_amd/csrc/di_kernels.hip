// Direction-independent StefCal kernels for gfx950: scalar (n_corr = 1) and 2x2 Jones
// (n_corr = 4) gains.
//
// One persistent launch solves the whole batch of solution intervals.  Each workgroup
// pops an interval from a device work queue (intervals pre-sorted by decreasing size),
// keeps that interval's gains in LDS and runs every update of Sect. 3.1 on it:
//
//   pass   : lane <-> baseline b; the lane walks the interval's samples s (rows
//            s * n_bl + b are consecutive across lanes, so every load is coalesced) and
//            accumulates, in registers, both sides of the folded row (Eq. JJ:di):
//              antenna p:  y = m conj(g_q)        A_p += |y|^2,  c_p += conj(y) d
//              antenna q:  y' = conj(m) conj(g_p) A_q += |y'|^2, c_q += conj(y') conj(d)
//            (2x2: Y = M G_q^H, Z_p += Y Y^H, N_p += D Y^H and, with X = G_p M,
//             Z_q += X^H X, N_q += D^H X -- the operator-diagonal blocks of Eq. JHJ:pol
//             and the matching J^H D).  Gains are per-lane constants over s.
//   reduce : a segmented wavefront scan over lanes that share an antenna, then one LDS
//            atomic per run and value (baselines in p-major order share p across a
//            wavefront, so the p side costs ~1 atomic per wave instead of 64).
//   solve  : per antenna, in FP64: g = c / A (Eq. stefcal) or G = N Z^-1 (polarized
//            update, least-squares order); singular blocks keep their gain; the
//            GN value or the lambda = 1 average (Eq. stefcal-lambda-average) per the
//            schedule; FP64 relative-change norm for the convergence test.
//   final  : residual R = D - G_p M G_q^H (flagged rows 0) and chi^2 in FP64.
//
// Flags are applied by selection (a flagged row never enters a sum), so non-finite
// values under a flag cannot leak into the results.
#include "wcal_internal.h"

namespace {

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

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

// Sum of x over the workgroup; `red` holds >= blockDim/64 doubles.  Result valid in every
// thread.  Contains barriers: call from uniform control flow only.
__device__ double block_sum(double x, double* red) {
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
__device__ void fold_waves(float* acc, int n) {
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

// One interval pass over all (baseline, sample) rows; wavefront w accumulates into its
// own slice acc[w][na][NV] (and cnt[na] in MODE 1), so the later fold over wavefronts in
// fixed order makes every result bit-reproducible.  In MODE 1 also forms the residual, writes it when
// requested and returns this thread's chi^2 contribution.
template <int NC, int MODE>
__device__ double interval_pass(const DiArgs& a, int64_t off, int ns, const float2* G,
                                float* acc, int* cnt) {
    constexpr int NV = Nv<NC, MODE>::v;
    const int nbl = a.n_bl;
    const bool has_flags = a.flags != nullptr;
    const bool write_res = (MODE == 1) && a.residual != nullptr;
    double chi = 0.0;
    acc += (threadIdx.x / WAVE) * a.n_ant * NV;
    for (int b0 = 0; b0 < nbl; b0 += blockDim.x) {
        const int b = b0 + threadIdx.x;
        const bool act = b < nbl;
        const int p = act ? a.ant1[b] : -1;
        const int q = act ? a.ant2[b] : -1;
        float vp[NV], vq[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) { vp[i] = 0.f; vq[i] = 0.f; }
        int nrow = 0;
        if (act) {
            if constexpr (NC == 1) {
                const float2 gp = G[p], gq = G[q];
                const float gp2 = nrm(gp), gq2 = nrm(gq);
#pragma unroll 4
                for (int s = 0; s < ns; ++s) {
                    const int64_t row = off + (int64_t)s * nbl + b;
                    const float2 d = a.data[row];
                    const float2 m = a.model[row];
                    const bool fl = has_flags && a.flags[row] != 0;
                    if (!fl) {
                        const float m2 = nrm(m);
                        const float2 y = cmulc(m, gq);      // y_pq = m conj(g_q)
                        const float2 yq = cmul(m, gp);      // conj(y_qp) = m g_p
                        vp[0] += m2 * gq2;
                        vq[0] += m2 * gp2;
                        const float2 cp = ccmul(y, d);      // conj(y) d
                        const float2 cq = cmulc(yq, d);     // conj(y') conj(d)
                        vp[1] += cp.x; vp[2] += cp.y;
                        vq[1] += cq.x; vq[2] += cq.y;
                        if constexpr (MODE == 1) {
                            const float2 r = csub(d, cmul(gp, y));   // d - g_p m conj(g_q)
                            const float2 rp = ccmul(y, r);
                            const float2 rq = cmulc(yq, r);
                            vp[3] += rp.x; vp[4] += rp.y;
                            vq[3] += rq.x; vq[4] += rq.y;
                            chi += (double)nrm(r);
                            ++nrow;
                            if (write_res) a.residual[row] = r;
                        }
                    } else if (write_res) {
                        a.residual[row] = make_float2(0.f, 0.f);
                    }
                }
            } else {
                const J2 Gp{G[4 * p], G[4 * p + 1], G[4 * p + 2], G[4 * p + 3]};
                const J2 Gq{G[4 * q], G[4 * q + 1], G[4 * q + 2], G[4 * q + 3]};
#pragma unroll 2
                for (int s = 0; s < ns; ++s) {
                    const int64_t row = off + (int64_t)s * nbl + b;
                    const J2 D = load_j2(a.data, row);
                    const J2 M = load_j2(a.model, row);
                    const bool fl = has_flags && a.flags[row] != 0;
                    if (!fl) {
                        const J2 Y = mulH(M, Gq);    // Y_pq = M G_q^H
                        const J2 X = mul(Gp, M);     // X = G_p M = Y_qp^H
                        // Z_p += Y Y^H (Hermitian: z00, z11, z01)
                        vp[0] += nrm(Y.a) + nrm(Y.b);
                        vp[1] += nrm(Y.c) + nrm(Y.d);
                        {
                            const float2 z = cadd(cmulc(Y.a, Y.c), cmulc(Y.b, Y.d));
                            vp[2] += z.x; vp[3] += z.y;
                        }
                        // Z_q += X^H X
                        vq[0] += nrm(X.a) + nrm(X.c);
                        vq[1] += nrm(X.b) + nrm(X.d);
                        {
                            const float2 z = cadd(ccmul(X.a, X.b), ccmul(X.c, X.d));
                            vq[2] += z.x; vq[3] += z.y;
                        }
                        // N_p += D Y^H ; N_q += D^H X
                        const J2 Np = mulH(D, Y);
                        const J2 Nq = Hmul(D, X);
                        vp[4] += Np.a.x; vp[5] += Np.a.y; vp[6] += Np.b.x; vp[7] += Np.b.y;
                        vp[8] += Np.c.x; vp[9] += Np.c.y; vp[10] += Np.d.x; vp[11] += Np.d.y;
                        vq[4] += Nq.a.x; vq[5] += Nq.a.y; vq[6] += Nq.b.x; vq[7] += Nq.b.y;
                        vq[8] += Nq.c.x; vq[9] += Nq.c.y; vq[10] += Nq.d.x; vq[11] += Nq.d.y;
                        if constexpr (MODE == 1) {
                            const J2 R = jsub(D, mul(Gp, Y));   // D - G_p M G_q^H
                            const J2 Rp = mulH(R, Y);            // R Y^H
                            const J2 Rq = Hmul(R, X);            // R^H X
                            vp[12] += Rp.a.x; vp[13] += Rp.a.y; vp[14] += Rp.b.x; vp[15] += Rp.b.y;
                            vp[16] += Rp.c.x; vp[17] += Rp.c.y; vp[18] += Rp.d.x; vp[19] += Rp.d.y;
                            vq[12] += Rq.a.x; vq[13] += Rq.a.y; vq[14] += Rq.b.x; vq[15] += Rq.b.y;
                            vq[16] += Rq.c.x; vq[17] += Rq.c.y; vq[18] += Rq.d.x; vq[19] += Rq.d.y;
                            chi += (double)(nrm(R.a) + nrm(R.b) + nrm(R.c) + nrm(R.d));
                            ++nrow;
                            if (write_res) store_j2(a.residual, row, R);
                        }
                    } else if (write_res) {
                        const float2 z = make_float2(0.f, 0.f);
                        store_j2(a.residual, row, J2{z, z, z, z});
                    }
                }
            }
        }
        seg_add<NV>(p, vp, acc, NV);
        seg_add<NV>(q, vq, acc, NV);
        if constexpr (MODE == 1) {
            seg_add_int(p, nrow, cnt);
            seg_add_int(q, nrow, cnt);
        }
    }
    return chi;
}

// Residual pass with fixed gains; writes R (if requested) and returns this thread's chi^2.
template <int NC>
__device__ double residual_pass(const DiArgs& a, int64_t off, int ns, const float2* G) {
    const int nbl = a.n_bl;
    const bool has_flags = a.flags != nullptr;
    float2* res = a.residual;
    double chi = 0.0;
    for (int b = threadIdx.x; b < nbl; b += blockDim.x) {
        const int p = a.ant1[b], q = a.ant2[b];
        float part = 0.f;
        if constexpr (NC == 1) {
            const float2 gp = G[p], gq = G[q];
#pragma unroll 4
            for (int s = 0; s < ns; ++s) {
                const int64_t row = off + (int64_t)s * nbl + b;
                const bool fl = has_flags && a.flags[row] != 0;
                float2 r = make_float2(0.f, 0.f);
                if (!fl) {
                    r = csub(a.data[row], cmul(gp, cmulc(a.model[row], gq)));
                    part += nrm(r);
                }
                if (res) res[row] = r;
            }
        } else {
            const J2 Gp{G[4 * p], G[4 * p + 1], G[4 * p + 2], G[4 * p + 3]};
            const J2 Gq{G[4 * q], G[4 * q + 1], G[4 * q + 2], G[4 * q + 3]};
#pragma unroll 2
            for (int s = 0; s < ns; ++s) {
                const int64_t row = off + (int64_t)s * nbl + b;
                const bool fl = has_flags && a.flags[row] != 0;
                const float2 z = make_float2(0.f, 0.f);
                J2 R{z, z, z, z};
                if (!fl) {
                    R = jsub(load_j2(a.data, row), mul(Gp, mulH(load_j2(a.model, row), Gq)));
                    part += nrm(R.a) + nrm(R.b) + nrm(R.c) + nrm(R.d);
                }
                if (res) store_j2(res, row, R);
            }
        }
        chi += (double)part;
    }
    return chi;
}

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

struct Ctl {
    int k;
    int flag;
};

template <int NC>
__global__ void __launch_bounds__(256) di_solve_kernel(DiArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NV = Nv<NC, 0>::v;
    const int na = a.n_ant;
    float2* G = reinterpret_cast<float2*>(smem);
    float2* Gn = G + na * NC;
    float* acc = reinterpret_cast<float*>(Gn + na * NC);
    __shared__ double red[16];
    __shared__ int s_k;
    __shared__ int s_bad, s_sing;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_k = atomicAdd(a.queue, 1);
        __syncthreads();
        const int idx = s_k;
        if (idx >= a.n_int) break;
        const int k = a.order[idx];
        const int64_t off = a.row_off[k];
        const int ns = a.ns[k];
        float2* gk = a.gains + (int64_t)k * na * NC;
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = gk[i];
        uint32_t status = 0;
        int n_it = 0;
        const int nacc = na * NV * (int)(blockDim.x / WAVE);
        for (int it = 0; it < a.max_iter; ++it) {
            for (int i = threadIdx.x; i < nacc; i += blockDim.x) acc[i] = 0.f;
            if (threadIdx.x == 0) { s_bad = 0; s_sing = 0; }
            __syncthreads();
            interval_pass<NC, 0>(a, off, ns, G, acc, nullptr);
            __syncthreads();
            fold_waves(acc, na * NV);
            const bool avg = avg_step(it, a.schedule);
            double dsum = 0.0, nsum = 0.0;
            for (int ant = threadIdx.x; ant < na; ant += blockDim.x) {
                double gh[2 * NC];
                bool fin = true;
                const bool ok = gn_value<NC>(acc + ant * NV, G + ant * NC, gh, fin);
                if (!fin) s_bad = 1;
                if (!ok) s_sing = 1;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const float2 go = G[ant * NC + c];
                    double nr = gh[2 * c], ni = gh[2 * c + 1];
                    if (avg) { nr = 0.5 * (go.x + nr); ni = 0.5 * (go.y + ni); }
                    const float2 gn = make_float2((float)nr, (float)ni);
                    Gn[ant * NC + c] = gn;
                    const double dr = (double)gn.x - go.x, di = (double)gn.y - go.y;
                    dsum += dr * dr + di * di;
                    nsum += (double)gn.x * gn.x + (double)gn.y * gn.y;
                }
            }
            dsum = block_sum(dsum, red);
            nsum = block_sum(nsum, red);
            // block_sum ends with a barrier, so s_bad / s_sing are final here
            if (s_bad) { status |= WCAL_NONFINITE; break; }
            if (s_sing) status |= WCAL_SINGULAR_ANT;
            for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = Gn[i];
            n_it = it + 1;
            const double num = sqrt(dsum), den = sqrt(nsum);
            const double rel = den == 0.0 ? (num == 0.0 ? 0.0 : INFINITY) : num / den;
            __syncthreads();
            if (rel < a.tol) { status |= WCAL_CONVERGED; break; }
        }
        if (!(status & (WCAL_CONVERGED | WCAL_NONFINITE))) status |= WCAL_MAXITER;
        __syncthreads();
        double chi = 0.0;
        if (a.residual != nullptr || a.chi2 != nullptr) chi = residual_pass<NC>(a, off, ns, G);
        chi = block_sum(chi, red);
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) gk[i] = G[i];
        if (threadIdx.x == 0) {
            a.n_iter[k] = n_it;
            a.status[k] = status;
            if (a.chi2) a.chi2[k] = chi;
        }
    }
}

template <int NC>
__global__ void __launch_bounds__(256) di_accumulate_kernel(DiArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NV = Nv<NC, 1>::v;
    const int na = a.n_ant;
    float2* G = reinterpret_cast<float2*>(smem);
    float* acc = reinterpret_cast<float*>(G + na * NC);
    int* cnt = reinterpret_cast<int*>(acc + na * NV * (int)(blockDim.x / WAVE));
    __shared__ double red[16];
    __shared__ int s_k;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_k = atomicAdd(a.queue, 1);
        __syncthreads();
        const int idx = s_k;
        if (idx >= a.n_int) break;
        const int k = a.order[idx];
        const int64_t off = a.row_off[k];
        const int ns = a.ns[k];
        const float2* gk = a.gains_in + (int64_t)k * na * NC;
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = gk[i];
        for (int i = threadIdx.x; i < na * NV * (int)(blockDim.x / WAVE); i += blockDim.x) acc[i] = 0.f;
        for (int i = threadIdx.x; i < na; i += blockDim.x) cnt[i] = 0;
        __syncthreads();
        double chi = interval_pass<NC, 1>(a, off, ns, G, acc, cnt);
        chi = block_sum(chi, red);
        fold_waves(acc, na * NV);
        const int64_t o = (int64_t)k * na;
        for (int ant = threadIdx.x; ant < na; ant += blockDim.x) {
            const float* v = acc + ant * NV;
            if constexpr (NC == 1) {
                a.jhj[o + ant] = make_float2(v[0], 0.f);
                a.jhd[o + ant] = make_float2(v[1], v[2]);
                a.jhr[o + ant] = make_float2(v[3], v[4]);
            } else {
                float2* z = a.jhj + (o + ant) * 4;
                z[0] = make_float2(v[0], 0.f);
                z[1] = make_float2(v[2], v[3]);
                z[2] = make_float2(v[2], -v[3]);
                z[3] = make_float2(v[1], 0.f);
                float2* n = a.jhd + (o + ant) * 4;
                float2* r = a.jhr + (o + ant) * 4;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    n[c] = make_float2(v[4 + 2 * c], v[5 + 2 * c]);
                    r[c] = make_float2(v[12 + 2 * c], v[13 + 2 * c]);
                }
            }
            if (a.count) a.count[o + ant] = cnt[ant];
        }
        if (threadIdx.x == 0 && a.chi2) a.chi2[k] = chi;
    }
}

template <int NC>
__global__ void __launch_bounds__(256) di_residual_kernel(DiArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int na = a.n_ant;
    float2* G = reinterpret_cast<float2*>(smem);
    __shared__ double red[16];
    __shared__ int s_k;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_k = atomicAdd(a.queue, 1);
        __syncthreads();
        const int idx = s_k;
        if (idx >= a.n_int) break;
        const int k = a.order[idx];
        const float2* gk = a.gains_in + (int64_t)k * na * NC;
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = gk[i];
        __syncthreads();
        double chi = residual_pass<NC>(a, a.row_off[k], a.ns[k], G);
        chi = block_sum(chi, red);
        if (threadIdx.x == 0 && a.chi2) a.chi2[k] = chi;
    }
}

__global__ void reset_queue_kernel(int32_t* q) {
    if (threadIdx.x < 4) q[threadIdx.x] = 0;
}

int grid_for(const wcal_plan* plan, const void* fn, int block, size_t smem) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, smem) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (plan->wg_per_cu > 0 && plan->wg_per_cu < per_cu) per_cu = plan->wg_per_cu;
    int64_t g = (int64_t)per_cu * plan->n_cu;
    if (g > plan->prob.n_int) g = plan->prob.n_int;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

size_t di_smem_bytes(int n_ant, int nc, int mode, int block) {
    const size_t g = (size_t)n_ant * nc * sizeof(float2);
    const size_t nw = (size_t)block / WAVE;
    if (mode == 0) return 2 * g + nw * n_ant * (nc == 1 ? 3 : 12) * sizeof(float);
    if (mode == 1) return g + nw * n_ant * (nc == 1 ? 5 : 20) * sizeof(float) + (size_t)n_ant * sizeof(int);
    return g;
}

hipError_t launch_reset_queue(int32_t* q, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, q);
    return hipGetLastError();
}

template <typename K>
static hipError_t launch_persistent(const wcal_plan* plan, K kernel, const DiArgs& a, size_t smem,
                                    hipStream_t s) {
    hipError_t e = launch_reset_queue(a.queue, s);
    if (e != hipSuccess) return e;
    const int block = plan->block;
    const int grid = grid_for(plan, reinterpret_cast<const void*>(kernel), block, smem);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), smem, s, a);
    return hipGetLastError();
}

hipError_t launch_di_solve(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    const int nc = plan->prob.n_corr;
    const size_t smem = di_smem_bytes(plan->prob.n_ant, nc, 0, plan->block);
    return nc == 1 ? launch_persistent(plan, di_solve_kernel<1>, a, smem, s)
                   : launch_persistent(plan, di_solve_kernel<4>, a, smem, s);
}

hipError_t launch_di_accumulate(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    const int nc = plan->prob.n_corr;
    const size_t smem = di_smem_bytes(plan->prob.n_ant, nc, 1, plan->block);
    return nc == 1 ? launch_persistent(plan, di_accumulate_kernel<1>, a, smem, s)
                   : launch_persistent(plan, di_accumulate_kernel<4>, a, smem, s);
}

hipError_t launch_di_residual(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    const int nc = plan->prob.n_corr;
    const size_t smem = di_smem_bytes(plan->prob.n_ant, nc, 2, plan->block);
    return nc == 1 ? launch_persistent(plan, di_residual_kernel<1>, a, smem, s)
                   : launch_persistent(plan, di_residual_kernel<4>, a, smem, s);
}
