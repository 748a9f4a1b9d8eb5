// Direction-independent StefCal kernels for gfx950: scalar (n_corr = 1) and 2x2 Jones
// (n_corr = 4) gains, batched over many solution intervals (Sect. 2.3).
//
// Per-sample solve (WCAL_MODE_PASS): every update streams all samples of the interval.
// Each update is two launches:
//   pass   : a persistent kernel pops tiles (baselines x samples of one interval) from the
//            list of tiles whose interval is still iterating.  Lane <-> baseline; the lane
//            walks the tile's samples (rows s * n_bl + b are consecutive across lanes, so
//            loads are coalesced; several rows are in flight per lane) and accumulates the
//            gain-independent statistics of its baseline: scalar sum |m|^2 and
//            sum conj(m) d; 2x2 the outer products sum vec(M) vec(M)^H and
//            sum vec(D) vec(M)^H.  At the end of the baseline they are contracted with
//            the current gains into both sides of the folded row (Eq. JJ:di):
//              antenna p:  A_p += |g_q|^2 sum|m|^2,  c_p += g_q sum conj(m) d
//              antenna q:  A_q += |g_p|^2 sum|m|^2,  c_q += g_p conj(sum conj(m) d)
//            (2x2: Z_p += sum M W_q M^H with W_q = G_q^H G_q, N_p += sum D G_q M^H,
//             Z_q += sum M^H W_p M, N_q += sum D^H G_p M -- the operator-diagonal blocks
//             of Eq. JHJ:pol and J^H D), i.e. exactly sum Y Y^H and sum D Y^H with
//            Y = M G_q^H.  A segmented wavefront scan over lanes that share an antenna
//            feeds per-wavefront LDS slices, folded in fixed order into one per-tile
//            partial per antenna.
//   update : one workgroup per iterating interval folds its tiles' partials in tile
//            order (bit-reproducible), solves every antenna in FP64 -- g = c / A
//            (Eq. stefcal) or G = N Z^-1 (the least-squares order of the polarized
//            update) -- applies the GN value or the lambda = 1 average
//            (Eq. stefcal-lambda-average) per the schedule, evaluates the FP64 relative
//            change and, if the interval keeps iterating, appends its tiles to the next
//            list.  Singular blocks keep their gain.
// By default the two steps run inside one persistent launch (di_loop_kernel): workgroups take
// tiles from a ring (loop_ring.h); the workgroup that finishes the last tile of an interval's
// update folds the tiles' partials in tile order, applies the update and puts the interval's
// tiles back while it keeps iterating, so intervals advance independently and a solve is one
// launch however many updates its intervals need.  The sums are those of the two-launch form,
// bit for bit.
// Statistics solve (WCAL_MODE_STATS): the statistics above do not depend on the gains,
// so one pass stores them per baseline and one persistent launch iterates every interval
// on them (the gains factor out of the sum over samples, as in the cross-direction
// terms of Sect. 3.2.1).
// Both modes end with a tiled residual pass R = D - G_p M G_q^H (flagged rows 0) and
// chi^2 in FP64.  Flags are applied by selection, so non-finite values under a flag
// cannot leak into any sum.
#include "di_common.h"

#define LOOP_FN __device__ __forceinline__
#include "loop_ring.h"

using namespace wcal_dev;

namespace {

// Data and model of one row.
template <int NC> struct Vis;
template <> struct Vis<1> { float2 d, m; };
template <> struct Vis<4> { J2 D, M; };

template <int NC>
__device__ __forceinline__ Vis<NC> load_vis(const DiArgs& a, int64_t row) {
    if constexpr (NC == 1) return Vis<1>{a.data[row], a.model[row]};
    else return Vis<4>{load_j2(a.data, row), load_j2(a.model, row)};
}

// Gains of the two antennas of a baseline, constant over the interval's samples.
template <int NC> struct Pair;
template <> struct Pair<1> { float2 gp, gq; float gp2, gq2; };
template <> struct Pair<4> { J2 Gp, Gq; };

// Both folded rows of one stored row (Eq. JJ:di): the antenna-p terms into vp and the
// antenna-q terms into vq.  MODE 1 also forms the residual and J^H r.
template <int NC, int MODE, int NV>
__device__ __forceinline__ void row_work(const DiArgs& a, const Pair<NC>& g, const Vis<NC>& v, bool fl,
                                         int64_t row, bool write_res, float (&vp)[NV], float (&vq)[NV],
                                         double& chi, int& nrow) {
    if constexpr (NC == 1) {
        if (!fl) {
            const float m2 = nrm(v.m);
            const float2 y = cmulc(v.m, g.gq);      // y_pq = m conj(g_q)
            const float2 yq = cmul(v.m, g.gp);      // conj(y_qp) = m g_p
            vp[0] += m2 * g.gq2;
            vq[0] += m2 * g.gp2;
            const float2 cp = ccmul(y, v.d);        // conj(y) d
            const float2 cq = cmulc(yq, v.d);       // conj(y') conj(d)
            vp[1] += cp.x; vp[2] += cp.y;
            vq[1] += cq.x; vq[2] += cq.y;
            if constexpr (MODE == 1) {
                const float2 r = csub(v.d, cmul(g.gp, y));   // d - g_p m conj(g_q)
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
    } else {
        if (!fl) {
            const J2 Y = mulH(v.M, g.Gq);   // Y_pq = M G_q^H
            const J2 X = mul(g.Gp, v.M);    // X = G_p M = Y_qp^H
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
            const J2 Np = mulH(v.D, Y);
            const J2 Nq = Hmul(v.D, X);
            vp[4] += Np.a.x; vp[5] += Np.a.y; vp[6] += Np.b.x; vp[7] += Np.b.y;
            vp[8] += Np.c.x; vp[9] += Np.c.y; vp[10] += Np.d.x; vp[11] += Np.d.y;
            vq[4] += Nq.a.x; vq[5] += Nq.a.y; vq[6] += Nq.b.x; vq[7] += Nq.b.y;
            vq[8] += Nq.c.x; vq[9] += Nq.c.y; vq[10] += Nq.d.x; vq[11] += Nq.d.y;
            if constexpr (MODE == 1) {
                const J2 R = jsub(v.D, mul(g.Gp, Y));   // D - G_p M G_q^H
                const J2 Rp = mulH(R, Y);                // R Y^H
                const J2 Rq = Hmul(R, X);                // R^H X
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

// Rows whose loads are issued together before any of them is used (memory-level
// parallelism per lane).
// Rows whose loads are issued together before any of them is used; sized so that the
// accumulate kernel does not spill at its workgroup size.
template <int NC, int MODE> struct Unroll { static constexpr int u = NC == 1 ? (MODE ? 4 : 8) : (MODE ? 2 : 4); };

// One interval pass over all (baseline, sample) rows; wavefront w accumulates into its
// own slice acc[w][na][NV] (and cnt[na] in MODE 1), so the later fold over wavefronts in
// fixed order makes every result bit-reproducible.  In MODE 1 also forms the residual,
// writes it when requested and returns this thread's chi^2 contribution.
template <int NC, int MODE>
__device__ double interval_pass(const DiArgs& a, int64_t off, int ns, const float2* G,
                                float* acc, int* cnt) {
    constexpr int NV = Nv<NC, MODE>::v;
    constexpr int U = Unroll<NC, MODE>::u;
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
            Pair<NC> g;
            if constexpr (NC == 1) {
                g.gp = G[p]; g.gq = G[q]; g.gp2 = nrm(g.gp); g.gq2 = nrm(g.gq);
            } else {
                g.Gp = J2{G[4 * p], G[4 * p + 1], G[4 * p + 2], G[4 * p + 3]};
                g.Gq = J2{G[4 * q], G[4 * q + 1], G[4 * q + 2], G[4 * q + 3]};
            }
            const int64_t base = off + b;
            int s = 0;
            for (; s + U <= ns; s += U) {
                Vis<NC> v[U];
                bool fl[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t row = base + (int64_t)(s + u) * nbl;
                    v[u] = load_vis<NC>(a, row);
                    fl[u] = has_flags && a.flags[row] != 0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    row_work<NC, MODE, NV>(a, g, v[u], fl[u], base + (int64_t)(s + u) * nbl, write_res,
                                           vp, vq, chi, nrow);
            }
            for (; s < ns; ++s) {
                const int64_t row = base + (int64_t)s * nbl;
                const Vis<NC> v = load_vis<NC>(a, row);
                const bool fl = has_flags && a.flags[row] != 0;
                row_work<NC, MODE, NV>(a, g, v, fl, row, write_res, vp, vq, chi, nrow);
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


// Workgroup size of the one-pass accumulate kernel: scalar 1024 threads, 2x2 512.
template <int NC> struct AccBlock { static constexpr int v = NC == 1 ? 1024 : 512; };

template <int NC>
__global__ void __launch_bounds__(AccBlock<NC>::v) di_accumulate_kernel(DiArgs a) {
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
        const int idx = __builtin_amdgcn_readfirstlane(s_k);
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


// ------------------------------------------------------------------ tiled solve
constexpr int TB = 256;   // workgroup size of every tiled kernel

// Floats of the per-baseline statistics: scalar sum|m|^2, sum conj(m) d; 2x2 the Hermitian
// 4x4 sum vec(M) vec(M)^H (4 real diagonal + 6 complex upper entries) and the 4x4 complex
// sum vec(D) vec(M)^H.  vec index e = 2 i + k for entry (i, k) of a 2x2 matrix.
template <int NC> struct Ns { static constexpr int v = NC == 1 ? 3 : 48; };

// Rows in flight per lane: in the statistics pass (2x2 at two rows fits 160 VGPRs, three
// waves per SIMD, and measures faster than four rows at two waves) and in the residual pass.
template <int NC> struct UT { static constexpr int v = NC == 1 ? 8 : 2; };
template <int NC> struct UR { static constexpr int v = NC == 1 ? 8 : 4; };

template <int NC>
__device__ __forceinline__ void stat_add(float (&st)[Ns<NC>::v], const Vis<NC>& v) {
    if constexpr (NC == 1) {
        st[0] += nrm(v.m);
        const float2 t = ccmul(v.m, v.d);        // conj(m) d
        st[1] += t.x; st[2] += t.y;
    } else {
        const float2 M[4] = {v.M.a, v.M.b, v.M.c, v.M.d};
        const float2 D[4] = {v.D.a, v.D.b, v.D.c, v.D.d};
#pragma unroll
        for (int e = 0; e < 4; ++e) st[e] += nrm(M[e]);
        int u = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int f = e + 1; f < 4; ++f, ++u) {
                const float2 t = cmulc(M[e], M[f]);   // M_e conj(M_f)
                st[4 + 2 * u] += t.x; st[5 + 2 * u] += t.y;
            }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const float2 t = cmulc(D[e], M[f]);   // D_e conj(M_f)
                st[16 + 2 * (4 * e + f)] += t.x; st[17 + 2 * (4 * e + f)] += t.y;
            }
    }
}

// entry (e, f) of sum vec(M) vec(M)^H from the packed Hermitian storage
__device__ __forceinline__ float2 smm(const float* st, int e, int f) {
    if (e == f) return make_float2(st[e], 0.f);
    if (e < f) {
        const int u = e * (7 - e) / 2 + (f - e - 1);
        return make_float2(st[4 + 2 * u], st[5 + 2 * u]);
    }
    const int u = f * (7 - f) / 2 + (e - f - 1);
    return make_float2(st[4 + 2 * u], -st[5 + 2 * u]);
}
__device__ __forceinline__ float2 sdm(const float* st, int e, int f) {
    return make_float2(st[16 + 2 * (4 * e + f)], st[17 + 2 * (4 * e + f)]);
}

// Contract one baseline's statistics with the gains of its antennas: per-antenna
// contributions in the layout of gn_value (scalar: A, c; 2x2: z00, z11, z01, N).
template <int NC>
__device__ __forceinline__ void contract(const float (&st)[Ns<NC>::v], const Pair<NC>& g,
                                         float (&vp)[Nv<NC, 0>::v], float (&vq)[Nv<NC, 0>::v]) {
    if constexpr (NC == 1) {
        const float2 s = make_float2(st[1], st[2]);
        vp[0] = g.gq2 * st[0];
        vq[0] = g.gp2 * st[0];
        const float2 cp = cmul(g.gq, s);
        const float2 cq = cmulc(g.gp, s);
        vp[1] = cp.x; vp[2] = cp.y;
        vq[1] = cq.x; vq[2] = cq.y;
    } else {
        const float2 Gp[4] = {g.Gp.a, g.Gp.b, g.Gp.c, g.Gp.d};
        const float2 Gq[4] = {g.Gq.a, g.Gq.b, g.Gq.c, g.Gq.d};
        // W = G^H G
        float2 Wp[4], Wq[4];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                Wp[2 * k + l] = cadd(ccmul(Gp[k], Gp[l]), ccmul(Gp[2 + k], Gp[2 + l]));
                Wq[2 * k + l] = cadd(ccmul(Gq[k], Gq[l]), ccmul(Gq[2 + k], Gq[2 + l]));
            }
        float2 Zp[4], Zq[4], Np[4], Nq[4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                float2 zp = make_float2(0.f, 0.f), zq = zp, np = zp, nq = zp;
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int l = 0; l < 2; ++l) {
                        zp = cadd(zp, cmul(Wq[2 * k + l], smm(st, 2 * i + k, 2 * j + l)));
                        zq = cadd(zq, cmul(Wp[2 * k + l], smm(st, 2 * l + j, 2 * k + i)));
                        np = cadd(np, cmul(Gq[2 * k + l], sdm(st, 2 * i + k, 2 * j + l)));
                        nq = cadd(nq, cmulc(Gp[2 * k + l], sdm(st, 2 * k + i, 2 * l + j)));
                    }
                Zp[2 * i + j] = zp; Zq[2 * i + j] = zq; Np[2 * i + j] = np; Nq[2 * i + j] = nq;
            }
        vp[0] = Zp[0].x; vp[1] = Zp[3].x; vp[2] = Zp[1].x; vp[3] = Zp[1].y;
        vq[0] = Zq[0].x; vq[1] = Zq[3].x; vq[2] = Zq[1].x; vq[3] = Zq[1].y;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            vp[4 + 2 * c] = Np[c].x; vp[5 + 2 * c] = Np[c].y;
            vq[4 + 2 * c] = Nq[c].x; vq[5 + 2 * c] = Nq[c].y;
        }
    }
}

template <int NC>
__device__ __forceinline__ Pair<NC> pair_from(const float2* G, int p, int q) {
    Pair<NC> g;
    if constexpr (NC == 1) {
        g.gp = G[p]; g.gq = G[q]; g.gp2 = nrm(g.gp); g.gq2 = nrm(g.gq);
    } else {
        g.Gp = J2{G[4 * p], G[4 * p + 1], G[4 * p + 2], G[4 * p + 3]};
        g.Gq = J2{G[4 * q], G[4 * q + 1], G[4 * q + 2], G[4 * q + 3]};
    }
    return g;
}

// Contract the statistics of the lane's current baseline and add both sides into this
// wavefront's LDS slice.  Every lane of the wavefront must call this.
template <int NC>
__device__ __forceinline__ void flush_acc(int p, int q, float (&st)[Ns<NC>::v], const float2* G, float* acc) {
    constexpr int NVP = Nv<NC, 0>::v;
    float vp[NVP], vq[NVP];
    if (p >= 0) {
        contract<NC>(st, pair_from<NC>(G, p, q), vp, vq);
    } else {
#pragma unroll
        for (int i = 0; i < NVP; ++i) { vp[i] = 0.f; vq[i] = 0.f; }
    }
    seg_add<NVP>(p, vp, acc, NVP);
    seg_add<NVP>(q, vq, acc, NVP);
#pragma unroll
    for (int i = 0; i < Ns<NC>::v; ++i) st[i] = 0.f;
}

// Walk a tile: items j = r * S + s (baseline round r of blockDim lanes, sample s), UT rows
// in flight per lane.  At each new round the previous round's statistics are handed to
// `flush(key_b, p, q, st)`; every lane reaches every flush (round changes are uniform).
template <int NC, typename Flush>
__device__ __forceinline__ void tile_walk(const DiArgs& a, const Tile& T, Flush flush) {
    constexpr int U = UT<NC>::v;
    constexpr int NS = Ns<NC>::v;
    const int BS = blockDim.x;
    const int R = (T.b1 - T.b0 + BS - 1) / BS;
    const int S = T.s1 - T.s0;
    const int total = R * S;
    const int64_t off = a.row_off[T.k];
    const bool has_flags = a.flags != nullptr;
    float st[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) st[i] = 0.f;
    int cur_b = -1, cur_p = -1, cur_q = -1;
    int r = 0, s = T.s0;
    for (int j0 = 0; j0 < total; j0 += U) {
        Vis<NC> v[U];
        bool valid[U], use[U], nr[U];
        int pp[U], qq[U], bb[U];
        int rr = r, ss = s;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            nr[u] = ss == T.s0;
            const int b = T.b0 + rr * BS + (int)threadIdx.x;
            bb[u] = b;
            valid[u] = (j0 + u < total) && (b < T.b1);
            use[u] = false;
            pp[u] = -1; qq[u] = -1;
            if (valid[u]) {
                const int64_t row = off + (int64_t)ss * a.n_bl + b;
                v[u] = load_vis<NC>(a, row);
                use[u] = !(has_flags && a.flags[row] != 0);
                if (nr[u]) { pp[u] = a.ant1[b]; qq[u] = a.ant2[b]; }
            }
            if (++ss == T.s1) { ss = T.s0; ++rr; }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (j0 + u >= total) break;
            if (nr[u]) {
                if (j0 + u > 0) flush(cur_b, cur_p, cur_q, st);
                cur_b = valid[u] ? bb[u] : -1;
                cur_p = pp[u];
                cur_q = qq[u];
            }
            if (use[u]) stat_add<NC>(st, v[u]);
        }
        r = rr; s = ss;
    }
    if (total > 0) flush(cur_b, cur_p, cur_q, st);
}

// Residual rows of a tile with the gains in LDS; returns this lane's chi^2 share.
template <int NC>
__device__ double tile_residual(const DiArgs& a, const Tile& T, const float2* G) {
    constexpr int U = UR<NC>::v;
    const int BS = blockDim.x;
    const int R = (T.b1 - T.b0 + BS - 1) / BS;
    const int S = T.s1 - T.s0;
    const int total = R * S;
    const int64_t off = a.row_off[T.k];
    const bool has_flags = a.flags != nullptr;
    float2* res = a.residual;
    double chi = 0.0;
    float part = 0.f;
    Pair<NC> g{};
    int r = 0, s = T.s0;
    for (int j0 = 0; j0 < total; j0 += U) {
        Vis<NC> v[U];
        bool valid[U], use[U], nr[U];
        int pp[U], qq[U];
        int64_t rows[U];
        int rr = r, ss = s;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            nr[u] = ss == T.s0;
            const int b = T.b0 + rr * BS + (int)threadIdx.x;
            valid[u] = (j0 + u < total) && (b < T.b1);
            use[u] = false;
            pp[u] = 0; qq[u] = 0;
            rows[u] = off + (int64_t)ss * a.n_bl + b;
            if (valid[u]) {
                v[u] = load_vis<NC>(a, rows[u]);
                use[u] = !(has_flags && a.flags[rows[u]] != 0);
                if (nr[u]) { pp[u] = a.ant1[b]; qq[u] = a.ant2[b]; }
            }
            if (++ss == T.s1) { ss = T.s0; ++rr; }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (nr[u] && valid[u]) {
                g = pair_from<NC>(G, pp[u], qq[u]);
                chi += (double)part;
                part = 0.f;
            }
            if (!valid[u]) continue;
            if constexpr (NC == 1) {
                float2 rv = make_float2(0.f, 0.f);
                if (use[u]) {
                    rv = csub(v[u].d, cmul(g.gp, cmulc(v[u].m, g.gq)));
                    part += nrm(rv);
                }
                if (res) res[rows[u]] = rv;
            } else {
                const float2 z = make_float2(0.f, 0.f);
                J2 R2{z, z, z, z};
                if (use[u]) {
                    R2 = jsub(v[u].D, mul(g.Gp, mulH(v[u].M, g.Gq)));
                    part += nrm(R2.a) + nrm(R2.b) + nrm(R2.c) + nrm(R2.d);
                }
                if (res) store_j2(res, rows[u], R2);
            }
        }
        r = rr; s = ss;
    }
    return chi + (double)part;
}

// One update of an interval from its folded per-antenna sums acc[na][NVP] (LDS).
// G holds the current gains (LDS), Gn receives the candidate.  Returns 1 when the
// interval stops (converged or non-finite), 0 when it keeps iterating; on a non-finite
// sum G is left unchanged.  Contains barriers: call from uniform control flow.
template <int NC>
__device__ int update_step(const DiArgs& a, int it, const float* acc, float2* G, float2* Gn, double* red,
                           int* s_flags, uint32_t& status) {
    constexpr int NVP = Nv<NC, 0>::v;
    const int na = a.n_ant;
    if (threadIdx.x == 0) { s_flags[0] = 0; s_flags[1] = 0; }
    __syncthreads();
    const bool avg = avg_step(it, a.schedule);
    double dsum = 0.0, nsum = 0.0;
    for (int ant = threadIdx.x; ant < na; ant += blockDim.x) {
        double gh[2 * NC];
        bool fin = true;
        const bool ok = gn_value<NC>(acc + ant * NVP, G + ant * NC, gh, fin);
        if (!fin) s_flags[0] = 1;
        if (!ok) s_flags[1] = 1;
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
    const int bad = s_flags[0], sing = s_flags[1];
    if (bad) { status |= WCAL_NONFINITE; __syncthreads(); return 1; }
    if (sing) status |= WCAL_SINGULAR_ANT;
    for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = Gn[i];
    __syncthreads();
    const double num = sqrt(dsum), den = sqrt(nsum);
    const double rel = den == 0.0 ? (num == 0.0 ? 0.0 : INFINITY) : num / den;
    if (rel < a.tol) { status |= WCAL_CONVERGED; return 1; }
    return 0;
}

// Counters: ctr[it] pops of the pass at update it, ctr[QOFF + it] tiles listed for it.
__device__ __forceinline__ int qoff(const DiArgs& a) { return a.max_iter + 2; }

__global__ void __launch_bounds__(TB) di_init_kernel(DiArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.n_int) {
        a.status[i] = 0;
        a.n_iter[i] = 0;
        a.active[i] = 1;
        if (a.tri_cnt) a.tri_cnt[i] = 0;
    }
    if (i < 2 * (a.max_iter + 2)) a.ctr[i] = 0;
}

// Zero the work-queue counters only (the residual entry point has no per-interval state).
__global__ void __launch_bounds__(TB) di_zero_ctr_kernel(DiArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2 * (a.max_iter + 2)) a.ctr[i] = 0;
}

template <int NC>
__global__ void __launch_bounds__(TB) di_pass_kernel(DiArgs a, int it) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NVP = Nv<NC, 0>::v;
    const int na = a.n_ant;
    float2* G = reinterpret_cast<float2*>(smem);
    float* acc = reinterpret_cast<float*>(G + na * NC);
    __shared__ int s_t;
    const int nw = blockDim.x / WAVE;
    const int n = it == 0 ? a.ntiles : a.ctr[qoff(a) + it];
    // tiles are popped dynamically, so workgroups beyond the listed count have nothing to
    // take (after convergence every workgroup leaves without touching the queue)
    if ((int)blockIdx.x >= n) return;
    const int32_t* list = a.lists + (it & 1) * a.ntiles;
    float* myacc = acc + (threadIdx.x / WAVE) * na * NVP;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = atomicAdd(&a.ctr[it], 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_t);
        if (idx >= n) break;
        const int t = it == 0 ? idx : list[idx];
        const Tile T = a.tiles[t];
        const float2* gk = a.gains + (int64_t)T.k * na * NC;
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = gk[i];
        for (int i = threadIdx.x; i < nw * na * NVP; i += blockDim.x) acc[i] = 0.f;
        __syncthreads();
        tile_walk<NC>(a, T, [&](int, int p, int q, float (&st)[Ns<NC>::v]) {
            flush_acc<NC>(p, q, st, G, myacc);
        });
        __syncthreads();
        float* out = a.partial + (int64_t)t * na * NVP;
        for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
            float v = acc[i];
            for (int w = 1; w < nw; ++w) v += acc[w * na * NVP + i];
            out[i] = v;
        }
    }
}

// ------------------------------------------------------------------ triangle pass
// Scalar gains, baselines in the canonical order (all pairs p < q, p-major): the stored
// rows of one sample form the upper triangle of an n_ant x n_ant matrix, and the folded
// sums of Eq. JJ:di are its row sums (antenna p) and column sums (antenna q):
//   A_p += |g_q|^2 sum|m|^2,   c_p += g_q sum conj(m) d,
//   A_q += |g_p|^2 sum|m|^2,   c_q += g_p conj(sum conj(m) d).
// A unit is a block of whole rows p (at most 64).  A wavefront walks each row in chunks of
// 64 consecutive baselines (lane = q - p - 1 - 64 j), so it streams the triangle in storage
// order and every cache line is consumed by one wavefront.  The row sum builds up in the
// lanes over the row's chunks and is reduced once per row (row-shift DPP adds, then the four
// row totals); lane (p - p0) keeps it until the unit ends.  Within a chunk the q are
// distinct, so each lane adds its column terms to the wavefront's LDS slice directly; the
// slice is private to the wavefront and updated in program order.  Every sum runs in a fixed
// order, so the pass is bit-reproducible.

// x from the lane n below in the same row of 16 lanes (0 for the first n lanes of a row)
template <int N>
__device__ __forceinline__ float dpp_row_shr(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + N, 0xf, 0xf, true));
}

// In the rows of ROWS: lane 15 of the row before (row broadcast, CTRL 0x142) or lane 31
// (0x143); x itself in the other rows.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_row_bcast(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), CTRL, ROWS, 0xf, false));
}

// Sum over the 64 lanes, returned uniformly: (r0 + r1) + (r2 + r3) of the four 16-lane row
// sums r.  Call with every lane active.  Only lane 63 is read at the end; the rows a
// broadcast leaves out hold values nothing reads.
__device__ __forceinline__ float wave_total(float x) {
    x += dpp_row_shr<1>(x);
    x += dpp_row_shr<2>(x);
    x += dpp_row_shr<4>(x);
    x += dpp_row_shr<8>(x);                  // lane 16 r + 15 holds the sum of row r
    x += dpp_row_bcast<0x142, 0xa>(x);       // lane 31: r1 + r0, lane 63: r3 + r2
    x += dpp_row_bcast<0x143, 0xc>(x);       // lane 63: (r3 + r2) + (r1 + r0)
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

constexpr int TRI_U = 4;    // chunks in flight per lane (4 measured best of 2..16)

// One unit of a tile (samples [s0, s1) of interval k) into this wavefront's slice
// acc[na + 1][3]; G holds na + 1 gains.  Lanes past the end of a row load the row's last
// element (no extra memory traffic), contribute zeros, and add them to the spare slot na.
// S1: the tile holds one sample (T.s1 == T.s0 + 1, every channel of the bandpass): each entry
// is complete at once, so its sums need no state between chunks.
template <bool S1>
__device__ __forceinline__ void tri_unit(const DiArgs& a, const Tile& T, const TriUnit& U, const float2* G,
                                         float* acc) {
    const int na = a.n_ant;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t off = a.row_off[T.k];
    const bool has_flags = a.flags != nullptr;
    float ps0 = 0.f, ps1 = 0.f, ps2 = 0.f;    // this lane's share of the current row sum
    float pr0 = 0.f, pr1 = 0.f, pr2 = 0.f;    // row sums of row p0 + lane
    float m2 = 0.f, tr = 0.f, ti = 0.f;       // sum|m|^2, sum conj(m) d of the current entry
    int p = U.p0, j = 0, s = T.s0;
    while (p < U.p1) {
        float2 d[TRI_U], m[TRI_U];
        bool use[TRI_U], end_e[TRI_U], end_r[TRI_U];
        int pu[TRI_U], qu[TRI_U];
        int pp = p, jj = j, ss = s;
#pragma unroll
        for (int u = 0; u < TRI_U; ++u) {
            const bool in = pp < U.p1;
            const int pr = in ? pp : U.p1 - 1;          // a row that exists
            const int len = na - 1 - pr;                 // baselines of row pr
            const int c = 64 * jj + lane;                // position in the row
            const bool valid = in && c < len;
            const int cc = valid ? c : len - 1;
            const int64_t base = off + (int64_t)ss * a.n_bl + (int64_t)pr * na - (int64_t)pr * (pr + 1) / 2;
            d[u] = load_at(a.data + base, cc);
            m[u] = load_at(a.model + base, cc);
            use[u] = valid && !(has_flags && load_at(a.flags + base, cc) != 0);
            pu[u] = pr;
            qu[u] = valid ? pr + 1 + c : na;
            if constexpr (S1) {
                end_e[u] = in;
                end_r[u] = in && 64 * (jj + 1) >= len;
                if (in && 64 * (++jj) >= len) { jj = 0; ++pp; }
            } else {
                end_e[u] = in && ss + 1 == T.s1;
                end_r[u] = end_e[u] && 64 * (jj + 1) >= len;
                if (in && ++ss == T.s1) {
                    ss = T.s0;
                    if (64 * (++jj) >= len) { jj = 0; ++pp; }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < TRI_U; ++u) {
            if constexpr (S1) {
                const float2 t = ccmul(m[u], d[u]);     // conj(m) d
                m2 = use[u] ? nrm(m[u]) : 0.f;
                tr = use[u] ? t.x : 0.f;
                ti = use[u] ? t.y : 0.f;
            } else if (use[u]) {
                m2 += nrm(m[u]);
                const float2 t = ccmul(m[u], d[u]);     // conj(m) d
                tr += t.x;
                ti += t.y;
            }
            if (end_e[u]) {                             // entry (pu, qu) complete: contract
                const float2 gp = G[pu[u]];
                const float2 gq = G[qu[u]];
                const float2 sv = make_float2(tr, ti);
                const float2 cp = cmul(gq, sv);
                const float2 cq = cmulc(gp, sv);        // g_p conj(s)
                ps0 += nrm(gq) * m2;
                ps1 += cp.x;
                ps2 += cp.y;
                float* dq = acc + qu[u] * 3;
                dq[0] += nrm(gp) * m2;
                dq[1] += cq.x;
                dq[2] += cq.y;
                m2 = 0.f; tr = 0.f; ti = 0.f;
            }
            if (end_r[u]) {                             // row pu complete: reduce its sum
                const float t0 = wave_total(ps0);
                const float t1 = wave_total(ps1);
                const float t2 = wave_total(ps2);
                if (lane == pu[u] - U.p0) { pr0 = t0; pr1 = t1; pr2 = t2; }
                ps0 = 0.f; ps1 = 0.f; ps2 = 0.f;
            }
        }
        p = pp; j = jj; s = ss;
    }
    if (lane < U.p1 - U.p0) {
        float* dst = acc + (U.p0 + lane) * 3;
        dst[0] += pr0; dst[1] += pr1; dst[2] += pr2;
    }
}

// Paired rows (plans that pack rows; n_ant >= TRI_PAIR_MIN): packed row r holds triangle row b = n_ant - 2 - r
// followed by row r, n_ant entries in all (row r alone when b == r), so every chunk but the
// last of the middle row is full.  A lane's entry is in row b or row r; each row's sum builds
// up in its own lane share (ra0..2, rb0..2), both reduced when the packed row ends; lane
// 2 (r - p0) keeps row r's total and lane 2 (r - p0) + 1 row b's.  With n_ant >= 127 the two
// rows of a chunk never share a column antenna, so the column read-modify-writes of a chunk
// stay distinct.  The unit's [p0, p1) counts packed rows.
__device__ __forceinline__ void tri_unit_paired(const DiArgs& a, const Tile& T, const TriUnit& U, const float2* G,
                                                float* acc) {
    const int na = a.n_ant;
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t off = a.row_off[T.k];
    const bool has_flags = a.flags != nullptr;
    float ra0 = 0.f, ra1 = 0.f, ra2 = 0.f;    // this lane's share of row r's sum
    float rb0 = 0.f, rb1 = 0.f, rb2 = 0.f;    // and of row b's
    float pr0 = 0.f, pr1 = 0.f, pr2 = 0.f;    // totals of the unit's row 2 (r - p0) + (lane & 1)
    float m2 = 0.f, tr = 0.f, ti = 0.f;       // sum|m|^2, sum conj(m) d of the current entry
    int r = U.p0, j = 0, s = T.s0;
    while (r < U.p1) {
        float2 d[TRI_U], m[TRI_U];
        bool use[TRI_U], inb[TRI_U], end_e[TRI_U], end_r[TRI_U];
        int pu[TRI_U], qu[TRI_U], ru[TRI_U];
        int rr = r, jj = j, ss = s;
#pragma unroll
        for (int u = 0; u < TRI_U; ++u) {
            const bool in = rr < U.p1;
            const int ra = in ? rr : U.p1 - 1;           // a packed row that exists
            const int rb = na - 2 - ra;
            const int la = na - 1 - ra, lb = rb > ra ? ra + 1 : 0;
            const int x = 64 * jj + lane;                // position in the packed row
            const bool valid = in && x < la + lb;
            const bool ib = x < lb;
            const int prow = ib ? rb : ra, c = ib ? x : x - lb;
            const int64_t rowbase = off + (int64_t)ss * a.n_bl;
            const int64_t ba = rowbase + (int64_t)ra * na - (int64_t)ra * (ra + 1) / 2;
            const int64_t bb = rowbase + (int64_t)rb * na - (int64_t)rb * (rb + 1) / 2;
            const int64_t at = valid ? (ib ? bb : ba) + c : ba + la - 1;   // else row r's last element
            d[u] = a.data[at];
            m[u] = a.model[at];
            use[u] = valid && !(has_flags && a.flags[at] != 0);
            inb[u] = valid && ib;
            pu[u] = valid ? prow : ra;
            qu[u] = valid ? prow + 1 + c : na;
            ru[u] = ra;
            end_e[u] = in && ss + 1 == T.s1;
            end_r[u] = end_e[u] && 64 * (jj + 1) >= la + lb;
            if (in && ++ss == T.s1) {
                ss = T.s0;
                if (64 * (++jj) >= la + lb) { jj = 0; ++rr; }
            }
        }
#pragma unroll
        for (int u = 0; u < TRI_U; ++u) {
            if (use[u]) {
                m2 += nrm(m[u]);
                const float2 t = ccmul(m[u], d[u]);     // conj(m) d
                tr += t.x;
                ti += t.y;
            }
            if (end_e[u]) {                             // entry (pu, qu) complete: contract
                const float2 gp = G[pu[u]];
                const float2 gq = G[qu[u]];
                const float2 sv = make_float2(tr, ti);
                const float2 cp = cmul(gq, sv);
                const float2 cq = cmulc(gp, sv);        // g_p conj(s)
                const float c0 = nrm(gq) * m2;
                if (inb[u]) { rb0 += c0; rb1 += cp.x; rb2 += cp.y; }
                else { ra0 += c0; ra1 += cp.x; ra2 += cp.y; }
                float* dq = acc + qu[u] * 3;
                dq[0] += nrm(gp) * m2;
                dq[1] += cq.x;
                dq[2] += cq.y;
                m2 = 0.f; tr = 0.f; ti = 0.f;
            }
            if (end_r[u]) {                             // packed row complete: reduce both sums
                const float a0 = wave_total(ra0), a1 = wave_total(ra1), a2 = wave_total(ra2);
                const float b0 = wave_total(rb0), b1 = wave_total(rb1), b2 = wave_total(rb2);
                const int slot = 2 * (ru[u] - U.p0);
                if (lane == slot) { pr0 = a0; pr1 = a1; pr2 = a2; }
                if (lane == slot + 1) { pr0 = b0; pr1 = b1; pr2 = b2; }
                ra0 = 0.f; ra1 = 0.f; ra2 = 0.f;
                rb0 = 0.f; rb1 = 0.f; rb2 = 0.f;
            }
        }
        r = rr; j = jj; s = ss;
    }
    if (lane < 2 * (U.p1 - U.p0)) {
        const int rw = U.p0 + (lane >> 1), rbw = na - 2 - rw;
        const int p = (lane & 1) ? rbw : rw;
        if (!((lane & 1) && rbw <= rw)) {             // a middle row has no partner
            float* dst = acc + p * 3;
            dst[0] += pr0; dst[1] += pr1; dst[2] += pr2;
        }
    }
}

template <int NC>
__device__ void finish_interval(const DiArgs& a, int it, int k, int t0, int t1, const float* acc, float2* G,
                                float2* Gn, double* red, int* s_flags, int* s_pos);

// FUSED: every interval is one tile, so the workgroup that sums a tile holds its interval's
// complete sums and applies the update itself (no update launch).  When few intervals are
// listed (the last updates, or a small batch), each is shared by S = min(4, grid / listed)
// workgroups, S chosen per launch from the listed count, so full passes keep S = 1: task
// (i, part) walks units b0 + part nw + w + j S nw of the i-th listed tile, folds its wavefront
// slices into partial (i, part) and counts itself in tri_cnt[i]; the workgroup that arrives
// last folds the S partials in part order, applies the update and clears the counter.  The
// sums keep a fixed order for a given S, so a solve is bit-reproducible; an interval's
// rounding can depend on how many others are still listed.  Alone on one workgroup, an
// interval of the bandpass takes ~45 us (a wavefront's 80 chunks at four in flight), which set
// the length of the last updates.
// Workgroup of the triangle pass: eight wavefronts walk an interval's units (three workgroups
// per CU at its 58 VGPRs).  Against four wavefronts, the tail updates, in which a few intervals
// are left and each runs on one workgroup, finish sooner, and full passes lose nothing
// (bandpass_na256 solve 6.45-6.60 -> 6.39 ms); six and twelve wavefronts measured slower.
constexpr int TRI_TB = 512;
constexpr int TRI_SPLIT_MAX = 4;
template <bool FUSED>
__global__ void __launch_bounds__(TRI_TB) di_tri_pass_kernel(DiArgs a, const TriUnit* __restrict__ units, int it) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NVP = Nv<1, 0>::v;
    const int na = a.n_ant;
    const int ns = (na + 1) * NVP;                  // slice: na antennas + the spare slot
    float2* G = reinterpret_cast<float2*>(smem);    // na + 1 (the last is 0)
    float* acc = reinterpret_cast<float*>(G + na + 1);
    float2* Gn = reinterpret_cast<float2*>(acc + (TRI_TB / WAVE) * ns);   // FUSED: candidate gains
    __shared__ double red[TRI_TB / WAVE];
    __shared__ int s_flags[2];
    __shared__ int s_pos;
    __shared__ int s_t;
    __shared__ int s_last;
    const int nw = blockDim.x / WAVE;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // wavefront-uniform
    const int n = it == 0 ? a.ntiles : a.ctr[qoff(a) + it];
    // workgroups per listed tile; the partials of n S tasks fit the plan's ntiles slots
    int S = 1;
    if (FUSED && a.tri_cnt && n > 0) S = max(1, min(TRI_SPLIT_MAX, min((int)gridDim.x / n, a.ntiles / n)));
    if ((int)blockIdx.x >= n * S) return;     // nothing to pop (see di_pass_kernel)
    const int32_t* list = a.lists + (it & 1) * a.ntiles;
    float* myacc = acc + w * ns;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = atomicAdd(&a.ctr[it], 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_t);
        if (idx >= n * S) break;
        const int ti = idx / S, part = idx - ti * S;
        const int t = it == 0 ? ti : list[ti];
        const Tile T = a.tiles[t];
        const float2* gk = a.gains + (int64_t)T.k * na;
        for (int i = threadIdx.x; i <= na; i += blockDim.x) G[i] = i < na ? gk[i] : make_float2(0.f, 0.f);
        for (int i = threadIdx.x; i < nw * ns; i += blockDim.x) acc[i] = 0.f;
        __syncthreads();
        const int u0 = T.b0 + part * nw + w, du = nw * S;
        if (a.tri_paired)
            for (int u = u0; u < T.b1; u += du) tri_unit_paired(a, T, units[u], G, myacc);
        else
            for (int u = u0; u < T.b1; u += du) {
                if (T.s1 - T.s0 == 1) tri_unit<true>(a, T, units[u], G, myacc);
                else tri_unit<false>(a, T, units[u], G, myacc);
            }
        __syncthreads();
        if constexpr (FUSED) {
            if (S > 1) {
                // This part's sums (wavefront slices folded in wavefront order) go out with
                // device-coherent stores; every wavefront waits until its stores are complete
                // before the workgroup counts itself, and the last workgroup reads the parts
                // with device-coherent loads.  (A device-scope fence would write back and
                // invalidate the XCD's whole L2 on every task.)
                float* out = a.partial + ((int64_t)ti * S + part) * na * NVP;
                for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
                    float v = acc[i];
                    for (int w2 = 1; w2 < nw; ++w2) v += acc[w2 * ns + i];
                    __hip_atomic_store(out + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (threadIdx.x == 0)
                    s_last = __hip_atomic_fetch_add(&a.tri_cnt[ti], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == S - 1;
                __syncthreads();
                if (!s_last) continue;          // another workgroup of the interval finishes it
                const float* in = a.partial + (int64_t)ti * S * na * NVP;
                for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
                    float v = __hip_atomic_load(in + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    for (int q = 1; q < S; ++q)
                        v += __hip_atomic_load(in + (int64_t)q * na * NVP + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    acc[i] = v;
                }
                if (threadIdx.x == 0) a.tri_cnt[ti] = 0;
            } else {
                // fold the wavefront slices into the first, in wavefront order
                for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
                    float v = acc[i];
                    for (int w2 = 1; w2 < nw; ++w2) v += acc[w2 * ns + i];
                    acc[i] = v;
                }
            }
            __syncthreads();
            finish_interval<1>(a, it, T.k, t, t + 1, acc, G, Gn, red, s_flags, &s_pos);
        } else {
            float* out = a.partial + (int64_t)t * na * NVP;
            for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
                float v = acc[i];
                for (int w2 = 1; w2 < nw; ++w2) v += acc[w2 * ns + i];
                out[i] = v;
            }
        }
    }
}

// Update `it` of interval k from its folded sums acc[na][NVP] (LDS): solve, schedule and
// convergence (update_step), write the gains, the status, the update count and the
// activity, and list the interval's tiles [t0, t1) for the next update if it keeps
// iterating.  Every thread of the workgroup must call this.
template <int NC>
__device__ void finish_interval(const DiArgs& a, int it, int k, int t0, int t1, const float* acc, float2* G,
                                float2* Gn, double* red, int* s_flags, int* s_pos) {
    const int na = a.n_ant;
    float2* gk = a.gains + (int64_t)k * na * NC;
    uint32_t status = 0;
    const int stop = update_step<NC>(a, it, acc, G, Gn, red, s_flags, status);
    bool finished = stop != 0;
    if (!(status & WCAL_NONFINITE)) {
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) gk[i] = G[i];
    }
    if (!finished && it + 1 >= a.max_iter) {
        status |= WCAL_MAXITER;
        finished = true;
    }
    if (threadIdx.x == 0) {
        a.status[k] |= status;
        if (!(status & WCAL_NONFINITE)) a.n_iter[k] = it + 1;
        if (finished) a.active[k] = 0;
        else *s_pos = atomicAdd(&a.ctr[qoff(a) + it + 1], t1 - t0);
    }
    if (!finished) {
        __syncthreads();
        int32_t* next = a.lists + ((it + 1) & 1) * a.ntiles;
        for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) next[*s_pos + i] = t0 + i;
    }
}

template <int NC>
__global__ void __launch_bounds__(TB) di_update_kernel(DiArgs a, int it) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NVP = Nv<NC, 0>::v;
    const int k = blockIdx.x;
    if (!a.active[k]) return;
    const int na = a.n_ant;
    float2* G = reinterpret_cast<float2*>(smem);
    float2* Gn = G + na * NC;
    float* acc = reinterpret_cast<float*>(Gn + na * NC);
    __shared__ double red[TB / WAVE];
    __shared__ int s_flags[2];
    __shared__ int s_pos;
    float2* gk = a.gains + (int64_t)k * na * NC;
    for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = gk[i];
    const int t0 = a.tile_off[k], t1 = a.tile_off[k + 1];
    for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
        float v = 0.f;
        for (int t = t0; t < t1; ++t) v += a.partial[(int64_t)t * na * NVP + i];
        acc[i] = v;
    }
    __syncthreads();
    finish_interval<NC>(a, it, k, t0, t1, acc, G, Gn, red, s_flags, &s_pos);
}

template <int NC>
__global__ void __launch_bounds__(TB) di_resid_kernel(DiArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int na = a.n_ant;
    float2* G = reinterpret_cast<float2*>(smem);
    __shared__ double red[TB / WAVE];
    __shared__ int s_t;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = atomicAdd(&a.ctr[2 * (a.max_iter + 2) - 1], 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_t);
        if (t >= a.ntiles) break;
        const Tile T = a.tiles[t];
        const float2* gk = a.gains_in + (int64_t)T.k * na * NC;
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = gk[i];
        __syncthreads();
        double chi = tile_residual<NC>(a, T, G);
        chi = block_sum(chi, red);
        if (threadIdx.x == 0) a.chi_part[t] = chi;
    }
}

__global__ void __launch_bounds__(TB) di_chi2_kernel(DiArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_int || !a.chi2) return;
    double c = 0.0;
    for (int t = a.tile_off[k]; t < a.tile_off[k + 1]; ++t) c += a.chi_part[t];
    a.chi2[k] = c;
}

// Statistics pass: the statistics of every baseline over all samples of its interval,
// stored structure-of-arrays per interval: stats[(k * NS + i) * n_bl + b].
template <int NC>
__global__ void __launch_bounds__(TB) di_stats_kernel(DiArgs a, const Tile* stiles, int nst) {
    constexpr int NS = Ns<NC>::v;
    __shared__ int s_t;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = atomicAdd(&a.ctr[0], 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_t);
        if (t >= nst) break;
        const Tile T = stiles[t];
        float* base = a.stats + (int64_t)T.k * NS * a.n_bl;
        tile_walk<NC>(a, T, [&](int b, int, int, float (&st)[NS]) {
            if (b >= 0) {
#pragma unroll
                for (int i = 0; i < NS; ++i) base[(int64_t)i * a.n_bl + b] = st[i];
            }
#pragma unroll
            for (int i = 0; i < NS; ++i) st[i] = 0.f;
        });
    }
}

// Iterate every interval on its stored statistics (one workgroup per interval, popped
// from a queue in decreasing-size order); per update the cost is O(n_bl), independent of
// the number of samples.
template <int NC>
__global__ void __launch_bounds__(TB) di_solve_stats_kernel(DiArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NVP = Nv<NC, 0>::v;
    constexpr int NS = Ns<NC>::v;
    const int na = a.n_ant;
    const int nw = blockDim.x / WAVE;
    float2* G = reinterpret_cast<float2*>(smem);
    float2* Gn = G + na * NC;
    float* acc = reinterpret_cast<float*>(Gn + na * NC);
    float* myacc = acc + (threadIdx.x / WAVE) * na * NVP;
    __shared__ double red[TB / WAVE];
    __shared__ int s_flags[2];
    __shared__ int s_k;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_k = atomicAdd(&a.ctr[1], 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_k);
        if (idx >= a.n_int) break;
        const int k = a.order[idx];
        float2* gk = a.gains + (int64_t)k * na * NC;
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) G[i] = gk[i];
        const float* base = a.stats + (int64_t)k * NS * a.n_bl;
        uint32_t status = 0;
        int n_it = 0;
        for (int it = 0; it < a.max_iter; ++it) {
            for (int i = threadIdx.x; i < nw * na * NVP; i += blockDim.x) acc[i] = 0.f;
            __syncthreads();
            for (int b0 = 0; b0 < a.n_bl; b0 += blockDim.x) {
                const int b = b0 + threadIdx.x;
                const bool act = b < a.n_bl;
                float st[NS];
#pragma unroll
                for (int i = 0; i < NS; ++i) st[i] = act ? base[(int64_t)i * a.n_bl + b] : 0.f;
                flush_acc<NC>(act ? a.ant1[b] : -1, act ? a.ant2[b] : -1, st, G, myacc);
            }
            __syncthreads();
            fold_waves(acc, na * NVP);
            const int stop = update_step<NC>(a, it, acc, G, Gn, red, s_flags, status);
            if (status & WCAL_NONFINITE) break;
            n_it = it + 1;
            if (stop) break;
        }
        if (!(status & (WCAL_CONVERGED | WCAL_NONFINITE))) status |= WCAL_MAXITER;
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) gk[i] = G[i];
        if (threadIdx.x == 0) {
            a.n_iter[k] = n_it;
            a.status[k] = status;
        }
    }
}

// ------------------------------------------------------------------ device-side iteration loop
// Agent-scope atomics for the ring of loop_ring.h.  The ring's waits poll with relaxed loads
// and take the acquire fence once, when the awaited word has arrived.
struct DevOps {
    __device__ int64_t add64(int64_t* p, int64_t v) {
        return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ int32_t add32_acq_rel(int32_t* p, int32_t v) {
        return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ uint64_t load64(uint64_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
    __device__ void store64_release(uint64_t* p, uint64_t v) {
        __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ void store64_relaxed(uint64_t* p, uint64_t v) {
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ int32_t load32(int32_t* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ void store32(int32_t* p, int32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ int64_t now() { return (int64_t)wall_clock64(); }
    __device__ void pause() { __builtin_amdgcn_s_sleep(2); }
};

// Values one workgroup of the loop writes and another reads in the same launch (the gains,
// the update count and status of an interval, the tiles' partial sums) move through
// agent-scope atomic loads and stores: those are coherent across the L2 caches of the XCDs,
// whereas a plain load may return a line that an L2 still holds from before the write.
__device__ __forceinline__ float2 ld_xwg(const float2* p) {
    const uint64_t v = __hip_atomic_load(const_cast<uint64_t*>(reinterpret_cast<const uint64_t*>(p)),
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}
__device__ __forceinline__ void st_xwg(float2* p, float2 x) {
    const uint64_t v = (uint64_t)__float_as_uint(x.x) | ((uint64_t)__float_as_uint(x.y) << 32);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_xwg(const float* p) {
    return __uint_as_float(__hip_atomic_load(const_cast<uint32_t*>(reinterpret_cast<const uint32_t*>(p)),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_xwg(float* p, float x) {
    __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __float_as_uint(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_xwg_int(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_xwg_int(T* p, T x) {
    __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The ring as the loop starts: HEAD 0, TAIL ntiles, every interval live, the first update's
// tiles in slots [0, ntiles), the other slots free for lap 0, every tile counter 0.
__global__ void __launch_bounds__(TB) loop_init_kernel(LoopRing q, int32_t ntiles, int32_t n_int) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < q.cap) q.ring[i] = i < ntiles ? ring_word(1, (uint32_t)i) : ring_word(0, 0);
    if (i < n_int) q.done[i] = 0;
    if (i == 0) {
        q.pos[LW_HEAD] = 0;
        q.pos[LW_TAIL] = ntiles;
        q.flag[LF_LIVE] = n_int;
        q.flag[LF_ABORT] = 0;
    }
}

// Update of interval k from its folded sums (acc, LDS) inside the loop: the update of
// finish_interval, then either the interval retires or its tiles [t0, t1) go back into the
// ring.  Every thread of the workgroup calls this.
template <int NC>
__device__ void loop_update(const DiArgs& a, const LoopRing& q, int k, int t0, int t1, const float* acc,
                            float2* G, float2* Gn, double* red, int* s_flags, int64_t* s_p0) {
    DevOps o;
    const int na = a.n_ant;
    const int it = ld_xwg_int(&a.n_iter[k]);     // updates applied so far
    float2* gk = a.gains + (int64_t)k * na * NC;
    uint32_t status = 0;
    const int stop = update_step<NC>(a, it, acc, G, Gn, red, s_flags, status);
    bool finished = stop != 0;
    if (!(status & WCAL_NONFINITE)) {
        for (int i = threadIdx.x; i < na * NC; i += blockDim.x) st_xwg(gk + i, G[i]);
    }
    if (!finished && it + 1 >= a.max_iter) {
        status |= WCAL_MAXITER;
        finished = true;
    }
    if (threadIdx.x == 0) {
        st_xwg_int(&a.status[k], ld_xwg_int(&a.status[k]) | status);
        if (!(status & WCAL_NONFINITE)) st_xwg_int(&a.n_iter[k], it + 1);
        if (finished) st_xwg_int(&a.active[k], 0);
    }
    if (finished) {
        if (threadIdx.x == 0) ring_retire(q, o);
        return;
    }
    // the new gains and the update count reach memory before any tile of the next update
    // can be taken
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *s_p0 = ring_reserve(q, o, t1 - t0);
    __syncthreads();
    const int64_t p0 = *s_p0;
    for (int i = threadIdx.x; i < t1 - t0; i += blockDim.x) ring_put(q, o, p0 + i, t0 + i);
}

// The whole PASS solve in one launch (see the top of the file).  TRI: the triangle pass of
// the canonical baseline order over the triangle tiles (scalar gains); else the tiled pass.
// LDS: gains G [na * NC] (TRI: na + 1, the last 0), the wavefront slices acc [nw][slice] with
// slice = na * NVP (TRI: (na + 1) * NVP), candidate gains Gn [na * NC].
// The 2x2 walk fits three waves per SIMD (at most 168 VGPRs), as the per-update pass does.
template <int NC> struct LoopWaves { static constexpr int v = NC == 4 ? 3 : 4; };

template <int NC, bool TRI>
__global__ void __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(LoopWaves<NC>::v, 8)))
di_loop_kernel(DiArgs a, LoopRing q, const TriUnit* __restrict__ units) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NVP = Nv<NC, 0>::v;
    const int na = a.n_ant;
    const int ng = TRI ? na + 1 : na * NC;
    const int sl = TRI ? (na + 1) * NVP : na * NVP;
    float2* G = reinterpret_cast<float2*>(smem);
    float* acc = reinterpret_cast<float*>(G + ng);
    float2* Gn = reinterpret_cast<float2*>(acc + (TB / WAVE) * sl);
    __shared__ double red[TB / WAVE];
    __shared__ int s_flags[2];
    __shared__ int s_t, s_last;
    __shared__ int64_t s_p0;
    const int nw = blockDim.x / WAVE;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // wavefront-uniform
    float* myacc = acc + w * sl;
    DevOps o;
    for (;;) {
        if (threadIdx.x == 0) s_t = ring_pop(q, o);
        __syncthreads();
        const int t = s_t;
        if (t < 0) break;
        const Tile T = a.tiles[t];
        const int k = T.k;
        const int t0 = a.tile_off[k], t1 = a.tile_off[k + 1];
        const float2* gk = a.gains + (int64_t)k * na * NC;
        for (int i = threadIdx.x; i < ng; i += blockDim.x) G[i] = (TRI && i == na) ? make_float2(0.f, 0.f) : ld_xwg(gk + i);
        for (int i = threadIdx.x; i < nw * sl; i += blockDim.x) acc[i] = 0.f;
        __syncthreads();
        if constexpr (TRI) {
            if (a.tri_paired)
                for (int u = T.b0 + w; u < T.b1; u += nw) tri_unit_paired(a, T, units[u], G, myacc);
            else
                for (int u = T.b0 + w; u < T.b1; u += nw) {
                    if (T.s1 - T.s0 == 1) tri_unit<true>(a, T, units[u], G, myacc);
                    else tri_unit<false>(a, T, units[u], G, myacc);
                }
        } else {
            tile_walk<NC>(a, T, [&](int, int p, int qq, float (&st)[Ns<NC>::v]) {
                flush_acc<NC>(p, qq, st, G, myacc);
            });
        }
        __syncthreads();
        if (t1 - t0 == 1) {
            // the interval's only tile: its sums are complete here (the wavefront slices
            // folded in wavefront order, as the partial of the two-launch form)
            for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
                float v = acc[i];
                for (int w2 = 1; w2 < nw; ++w2) v += acc[w2 * sl + i];
                acc[i] = v;
            }
            __syncthreads();
        } else {
            float* out = a.partial + (int64_t)t * na * NVP;
            for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
                float v = acc[i];
                for (int w2 = 1; w2 < nw; ++w2) v += acc[w2 * sl + i];
                st_xwg(out + i, v);
            }
            __threadfence();          // every thread's partial is in memory before the count
            __syncthreads();
            if (threadIdx.x == 0) s_last = ring_tile_done(q, o, k, t1 - t0);
            __syncthreads();
            if (!s_last) continue;
            // the update's last tile: every partial of the interval is visible (the count's
            // acquire); fold them in tile order
            for (int i = threadIdx.x; i < na * NVP; i += blockDim.x) {
                float v = 0.f;
                for (int tt = t0; tt < t1; ++tt) v += ld_xwg(a.partial + (int64_t)tt * na * NVP + i);
                acc[i] = v;
            }
            __syncthreads();
        }
        loop_update<NC>(a, q, k, t0, t1, acc, G, Gn, red, s_flags, &s_p0);
    }
}

// After the loop: an interval still marked active was cut off by an aborted wait.
__global__ void __launch_bounds__(TB) loop_end_kernel(DiArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < a.n_int && a.active[k]) a.status[k] |= WCAL_ABORTED;
}

__global__ void reset_queue_kernel(int32_t* q) {
    if (threadIdx.x < 4) q[threadIdx.x] = 0;
}

int grid_resident(const wcal_plan* plan, const void* fn, int block, size_t smem, int64_t work) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, smem) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (plan->wg_per_cu > 0 && plan->wg_per_cu < per_cu) per_cu = plan->wg_per_cu;
    int64_t g = (int64_t)per_cu * plan->n_cu;
    if (g > work) g = work;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

int di_nvp(int nc) { return nc == 1 ? Nv<1, 0>::v : Nv<4, 0>::v; }
int di_nstat(int nc) { return nc == 1 ? Ns<1>::v : Ns<4>::v; }

size_t di_accumulate_smem(int n_ant, int nc, int block) {
    const size_t g = (size_t)n_ant * nc * sizeof(float2);
    const size_t nw = (size_t)block / WAVE;
    return g + nw * n_ant * (nc == 1 ? 5 : 20) * sizeof(float) + (size_t)n_ant * sizeof(int);
}

static size_t pass_smem(int na, int nc) {
    return (size_t)na * nc * sizeof(float2) + (size_t)(TB / WAVE) * na * di_nvp(nc) * sizeof(float);
}
static size_t update_smem(int na, int nc) {
    return 2 * (size_t)na * nc * sizeof(float2) + (size_t)(TB / WAVE) * na * di_nvp(nc) * sizeof(float);
}

// The ring of the device-side loop in the plan's WS_LOOP region: 64 bytes of control words
// (two int64 positions, then LIVE and ABORT), the slots, the per-interval tile counters.
static LoopRing loop_ring_of(const wcal_plan* plan, int32_t ntiles) {
    char* base = reinterpret_cast<char*>(plan->d_loop);
    LoopRing q;
    q.pos = reinterpret_cast<int64_t*>(base);
    q.flag = reinterpret_cast<int32_t*>(base + 2 * sizeof(int64_t));
    q.ring = reinterpret_cast<uint64_t*>(base + 64);
    q.cap = (int64_t)LOOP_RING * ntiles;
    q.done = reinterpret_cast<int32_t*>(base + 64 + ws_round(sizeof(uint64_t) * (size_t)q.cap));
    q.limit = (int64_t)ntiles * plan->prob.max_iter;
    q.wait_ticks = plan->wait_ticks;
    return q;
}

hipError_t launch_reset_queue(int32_t* q, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, q);
    return hipGetLastError();
}

size_t kernel_static_lds(const void* fn) {
    hipFuncAttributes at{};
    return hipFuncGetAttributes(&at, fn) == hipSuccess ? at.sharedSizeBytes : (size_t)32 << 10;
}

template <int NC>
static hipError_t solve_nc(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    const int na = plan->prob.n_ant;
    prof_begin(plan, WCAL_K_OTHER, s);
    hipLaunchKernelGGL(di_init_kernel, dim3((std::max(a.n_int, 2 * (a.max_iter + 2)) + TB - 1) / TB), dim3(TB),
                       0, s, a);
    prof_end(plan, WCAL_K_OTHER, s);
    const size_t us = update_smem(na, NC);
    if (di_stats_solve(plan)) {
        const int g1 = grid_resident(plan, reinterpret_cast<const void*>(di_stats_kernel<NC>), TB, 0, plan->nstiles);
        prof_begin(plan, WCAL_K_STATS, s);
        hipLaunchKernelGGL(di_stats_kernel<NC>, dim3(g1), dim3(TB), 0, s, a, (const Tile*)plan->d_stiles,
                           plan->nstiles);
        prof_end(plan, WCAL_K_STATS, s);
        const int g2 = grid_resident(plan, reinterpret_cast<const void*>(di_solve_stats_kernel<NC>), TB, us,
                                     a.n_int);
        prof_begin(plan, WCAL_K_SOLVE_STATS, s);
        hipLaunchKernelGGL(di_solve_stats_kernel<NC>, dim3(g2), dim3(TB), us, s, a);
        prof_end(plan, WCAL_K_SOLVE_STATS, s);
    } else if (plan->loop) {
        // one persistent launch iterates every interval (triangle tiles when the plan uses the
        // triangle pass; the residual below keeps the row tiles)
        DiArgs at = a;
        const bool tri = NC == 1 && plan->tri;
        if (tri) {
            at.tiles = plan->d_ttiles;
            at.tile_off = plan->d_ttile_off;
            at.ntiles = plan->nttiles;
        }
        const LoopRing q = loop_ring_of(plan, at.ntiles);
        hipLaunchKernelGGL(loop_init_kernel, dim3((unsigned)((q.cap + TB - 1) / TB)), dim3(TB), 0, s, q, at.ntiles,
                           a.n_int);
        const size_t ls = tri ? (size_t)(na + 1) * sizeof(float2) + (size_t)(TB / WAVE) * (na + 1) * 3 * sizeof(float) +
                                    (size_t)na * sizeof(float2)
                              : update_smem(na, NC);
        const void* fn = tri ? reinterpret_cast<const void*>(di_loop_kernel<1, true>)
                             : reinterpret_cast<const void*>(di_loop_kernel<NC, false>);
        const int gl = grid_resident(plan, fn, TB, ls, at.ntiles);
        prof_begin(plan, WCAL_K_PASS, s);
        if (tri)
            hipLaunchKernelGGL((di_loop_kernel<1, true>), dim3(gl), dim3(TB), ls, s, at, q, (const TriUnit*)plan->d_units);
        else
            hipLaunchKernelGGL((di_loop_kernel<NC, false>), dim3(gl), dim3(TB), ls, s, at, q, (const TriUnit*)nullptr);
        prof_end(plan, WCAL_K_PASS, s);
        hipLaunchKernelGGL(loop_end_kernel, dim3((a.n_int + TB - 1) / TB), dim3(TB), 0, s, a);
    } else if (NC == 1 && plan->tri) {
        // pass and update over the triangle tiles; the residual below keeps the row tiles
        DiArgs at = a;
        at.tiles = plan->d_ttiles;
        at.tile_off = plan->d_ttile_off;
        at.ntiles = plan->nttiles;
        const bool fused = plan->nttiles == a.n_int;    // one tile per interval
        const size_t ps = (size_t)(na + 1) * sizeof(float2) + (size_t)(TRI_TB / WAVE) * (na + 1) * 3 * sizeof(float) +
                          (fused ? (size_t)na * sizeof(float2) : 0);
        const void* fn = fused ? reinterpret_cast<const void*>(di_tri_pass_kernel<true>)
                               : reinterpret_cast<const void*>(di_tri_pass_kernel<false>);
        // the fused pass may share a listed interval among up to TRI_SPLIT_MAX workgroups
        const int gp = grid_resident(plan, fn, TRI_TB, ps, (int64_t)at.ntiles * (fused ? TRI_SPLIT_MAX : 1));
        for (int it = 0; it < a.max_iter; ++it) {
            prof_begin(plan, WCAL_K_PASS, s);
            if (fused)
                hipLaunchKernelGGL(di_tri_pass_kernel<true>, dim3(gp), dim3(TRI_TB), ps, s, at, (const TriUnit*)plan->d_units, it);
            else
                hipLaunchKernelGGL(di_tri_pass_kernel<false>, dim3(gp), dim3(TRI_TB), ps, s, at, (const TriUnit*)plan->d_units, it);
            prof_end(plan, WCAL_K_PASS, s);
            if (!fused) {
                prof_begin(plan, WCAL_K_UPDATE, s);
                hipLaunchKernelGGL(di_update_kernel<1>, dim3(a.n_int), dim3(TB), us, s, at, it);
                prof_end(plan, WCAL_K_UPDATE, s);
            }
            if (watch_stop(plan, s, a.ctr + (a.max_iter + 2) + it + 1, it)) break;   // tiles listed for it + 1
        }
    } else {
        const size_t ps = pass_smem(na, NC);
        const int gp = grid_resident(plan, reinterpret_cast<const void*>(di_pass_kernel<NC>), TB, ps, a.ntiles);
        for (int it = 0; it < a.max_iter; ++it) {
            prof_begin(plan, WCAL_K_PASS, s);
            hipLaunchKernelGGL(di_pass_kernel<NC>, dim3(gp), dim3(TB), ps, s, a, it);
            prof_end(plan, WCAL_K_PASS, s);
            prof_begin(plan, WCAL_K_UPDATE, s);
            hipLaunchKernelGGL(di_update_kernel<NC>, dim3(a.n_int), dim3(TB), us, s, a, it);
            prof_end(plan, WCAL_K_UPDATE, s);
            if (watch_stop(plan, s, a.ctr + (a.max_iter + 2) + it + 1, it)) break;   // tiles listed for it + 1
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.residual || a.chi2) {
        DiArgs r = a;
        r.gains_in = a.gains;
        const size_t rs = (size_t)na * NC * sizeof(float2);
        const int gr = grid_resident(plan, reinterpret_cast<const void*>(di_resid_kernel<NC>), TB, rs, a.ntiles);
        prof_begin(plan, WCAL_K_RESID, s);
        hipLaunchKernelGGL(di_resid_kernel<NC>, dim3(gr), dim3(TB), rs, s, r);
        prof_end(plan, WCAL_K_RESID, s);
        prof_begin(plan, WCAL_K_OTHER, s);
        hipLaunchKernelGGL(di_chi2_kernel, dim3((a.n_int + TB - 1) / TB), dim3(TB), 0, s, r);
        prof_end(plan, WCAL_K_OTHER, s);
    }
    return hipGetLastError();
}

// Scalar pass of update `it` that leaves the per-tile per-antenna sums in a.partial and
// applies no update: the triangle pass over the triangle tiles when the plan uses it, else
// the tiled pass.  Launches are timed on prof_plan's profiler.  Tiles are listed as the update kernels list them (all tiles for it = 0,
// a.lists / a.ctr after that).  Used by the smoothed solve, whose update needs the sums of
// neighbouring cells.
hipError_t launch_di_pass_partials(const wcal_plan* plan, const wcal_plan* prof_plan, const DiArgs& a, int it,
                                   hipStream_t s) {
    const int na = plan->prob.n_ant;
    prof_begin(prof_plan, WCAL_K_PASS, s);
    if (plan->tri) {
        DiArgs at = a;
        at.tiles = plan->d_ttiles;
        at.tile_off = plan->d_ttile_off;
        at.ntiles = plan->nttiles;
        const size_t ps = (size_t)(na + 1) * sizeof(float2) + (size_t)(TRI_TB / WAVE) * (na + 1) * 3 * sizeof(float);
        const int gp = grid_resident(plan, reinterpret_cast<const void*>(di_tri_pass_kernel<false>), TRI_TB, ps, at.ntiles);
        hipLaunchKernelGGL(di_tri_pass_kernel<false>, dim3(gp), dim3(TRI_TB), ps, s, at, (const TriUnit*)plan->d_units, it);
    } else {
        const size_t ps = pass_smem(na, 1);
        const int gp = grid_resident(plan, reinterpret_cast<const void*>(di_pass_kernel<1>), TB, ps, a.ntiles);
        hipLaunchKernelGGL(di_pass_kernel<1>, dim3(gp), dim3(TB), ps, s, a, it);
    }
    prof_end(prof_plan, WCAL_K_PASS, s);
    return hipGetLastError();
}

// The tile table launch_di_pass_partials works on: interval k owns tiles
// [off[k], off[k + 1]) of it.
const int32_t* di_pass_tile_off(const wcal_plan* plan) { return plan->tri ? plan->d_ttile_off : plan->d_tile_off; }
int32_t di_pass_ntiles(const wcal_plan* plan) { return plan->tri ? plan->nttiles : plan->ntiles; }

// Scalar residual rows of every tile with gains a.gains_in, chi^2 per tile in a.chi_part
// (the sums per interval are left to the caller).
hipError_t launch_di_resid_tiles(const wcal_plan* plan, const wcal_plan* prof_plan, const DiArgs& a, hipStream_t s) {
    const int na = plan->prob.n_ant;
    hipLaunchKernelGGL(di_zero_ctr_kernel, dim3((2 * (a.max_iter + 2) + TB - 1) / TB), dim3(TB), 0, s, a);
    const size_t rs = (size_t)na * sizeof(float2);
    const int gr = grid_resident(plan, reinterpret_cast<const void*>(di_resid_kernel<1>), TB, rs, a.ntiles);
    prof_begin(prof_plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(di_resid_kernel<1>, dim3(gr), dim3(TB), rs, s, a);
    prof_end(prof_plan, WCAL_K_RESID, s);
    return hipGetLastError();
}

hipError_t launch_di_solve(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    return plan->prob.n_corr == 1 ? solve_nc<1>(plan, a, s) : solve_nc<4>(plan, a, s);
}

template <int NC>
static hipError_t residual_nc(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    const int na = plan->prob.n_ant;
    // status / n_iter are not outputs here: only the counters are reset
    hipLaunchKernelGGL(di_zero_ctr_kernel, dim3((2 * (a.max_iter + 2) + TB - 1) / TB), dim3(TB), 0, s, a);
    const size_t rs = (size_t)na * NC * sizeof(float2);
    const int gr = grid_resident(plan, reinterpret_cast<const void*>(di_resid_kernel<NC>), TB, rs, a.ntiles);
    prof_begin(plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(di_resid_kernel<NC>, dim3(gr), dim3(TB), rs, s, a);
    prof_end(plan, WCAL_K_RESID, s);
    hipLaunchKernelGGL(di_chi2_kernel, dim3((a.n_int + TB - 1) / TB), dim3(TB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_di_residual(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    return plan->prob.n_corr == 1 ? residual_nc<1>(plan, a, s) : residual_nc<4>(plan, a, s);
}

template <int NC>
static hipError_t accumulate_nc(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    hipError_t e = launch_reset_queue(a.queue, s);
    if (e != hipSuccess) return e;
    const int block = AccBlock<NC>::v;
    const size_t smem = di_accumulate_smem(plan->prob.n_ant, NC, block);
    const int grid = grid_resident(plan, reinterpret_cast<const void*>(di_accumulate_kernel<NC>), block, smem,
                                   plan->prob.n_int);
    hipLaunchKernelGGL(di_accumulate_kernel<NC>, dim3(grid), dim3(block), smem, s, a);
    return hipGetLastError();
}

hipError_t launch_di_accumulate(const wcal_plan* plan, const DiArgs& a, hipStream_t s) {
    return plan->prob.n_corr == 1 ? accumulate_nc<1>(plan, a, s) : accumulate_nc<4>(plan, a, s);
}
