// Receiver-conditioned radiance of RxGS on the device (Sec. 4.3.2 eqs.
// rx_enc, film, film_apply, transmittance, local, combined_local; App. E.2,
// E.5; Alg. 1 stage 2: rxcond.forward_batched, then eval_fle against the
// basis of the view centre's direction).
//
// Per render:
//   k_rxcond_gamma   receiver term of the global MLP's first layer (the
//                    Fourier encoding in FP64), once per receiver;
//   k_rxcond_global  the global MLP per (receiver, component): (1 + alpha,
//                    beta) for every channel -- O(L) per receiver;
//   k_rxcond_local   per MLP work item (view, 32 sorted positions, receivers):
//                    the 16 occupancy probes (FP64 positions, so each probe
//                    reads the voxel the definition names), the local MLP's
//                    layer 1 on the VALU, layer 2 on FP32 MFMA
//                    (v_mfma_f32_32x32x2f32, one pair per lane pair), layer 3
//                    per lane pair: (1 + alpha', beta') per channel;
//   k_rxcond_eval    per work item: the basis by the associated-Legendre
//                    recurrence, streamed component by component, reduced
//                    against the modulated coefficients, then the local
//                    modulation: the radiance of every (receiver, channel) row.
// Per upload: the occupancy grid (k_rc_bounds, k_rc_splat with exact
// integer sums, k_rc_finish) and the coefficients in walk order.
//
// Walk order.  The two lanes of a pair (lane halves h = 0, 1) split the
// components by the parity of |m|: half h walks m = h, h + 2, ..., and for
// each m the degrees l = m .. lmax, taking (l, +m) then (l, -m).  Coefficient
// rows and the global modulation are stored in this order (half 0's
// positions first), so each lane reads its half-row front to back.
#include "device_common.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace rxgs {

namespace {

constexpr int RC_H = RXGS_RXCOND_HIDDEN;
constexpr int RC_TAB = 13;          // (l, m) table side: lmax <= 12
constexpr int RC_CH_PASS = 8;       // channels accumulated per basis walk
constexpr double OCC_SCALE = 68719476736.0;   // 2^36: fixed-point scale of the log-transmission sums

struct RcBox {
    double lo[3], inv[3], vs[3];
};

// ---------------------------------------------------------------------------
// occupancy grid (App. E.5)

__device__ __forceinline__ unsigned ord_key(float f)
{
    const unsigned b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// componentwise min / max of the means as order-preserving keys
__global__ __launch_bounds__(BLOCK) void k_rc_bounds(const float *__restrict__ soa, int64_t K,
                                                     unsigned *__restrict__ out /* 6: min xyz, max xyz */)
{
    unsigned mn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, mx[3] = {0u, 0u, 0u};
    for (int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x; k < K; k += (int64_t)gridDim.x * BLOCK)
        for (int a = 0; a < 3; a++) {
            const unsigned key = ord_key(soa[a * K + k]);
            mn[a] = min(mn[a], key);
            mx[a] = max(mx[a], key);
        }
    for (int a = 0; a < 3; a++) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            mn[a] = min(mn[a], (unsigned)__shfl_xor((int)mn[a], o));
            mx[a] = max(mx[a], (unsigned)__shfl_xor((int)mx[a], o));
        }
    }
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; a++) {
            atomicMin(out + a, mn[a]);
            atomicMax(out + 3 + a, mx[a]);
        }
}

// One wave per Gaussian: every voxel centre within 2 sigma (sigma = the
// largest scale) adds log(1 - o exp(-d^2 / (2 sigma^2))) to its voxel, as an
// integer in units of 2^-36 (sums of integers do not depend on the order, so
// the grid is the same on every upload).  The voxel range and the 2 sigma
// test are evaluated in FP64 in the order the definition is written, so the
// set of voxels each Gaussian reaches is the definition's.
__global__ __launch_bounds__(BLOCK) void k_rc_splat(const float *__restrict__ soa, int64_t K, int G, RcBox box,
                                                    unsigned long long *__restrict__ acc)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / 64);
    for (int64_t k = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); k < K; k += nw) {
        const double p[3] = {(double)soa[k], (double)soa[K + k], (double)soa[2 * K + k]};
        double lsm = (double)soa[3 * K + k];
        lsm = fmax(lsm, (double)soa[4 * K + k]);
        lsm = fmax(lsm, (double)soa[5 * K + k]);
        const double sig = exp(lsm);
        const double o = 1.0 / (1.0 + exp(-(double)soa[10 * K + k]));
        const double r2 = 4.0 * sig * sig;
        int i0[3], n[3];
        bool empty = false;
        for (int a = 0; a < 3; a++) {
            int lo = (int)floor((p[a] - 2.0 * sig - box.lo[a]) / box.vs[a]) - 1;
            int hi = (int)floor((p[a] + 2.0 * sig - box.lo[a]) / box.vs[a]) + 1;
            lo = max(lo, 0);
            hi = min(hi, G - 1);
            i0[a] = lo;
            n[a] = hi - lo + 1;
            empty |= n[a] <= 0;
        }
        if (empty) continue;
        const int64_t total = (int64_t)n[0] * n[1] * n[2];
        for (int64_t i = lane; i < total; i += 64) {
            const int ix = i0[0] + (int)(i % n[0]);
            const int iy = i0[1] + (int)((i / n[0]) % n[1]);
            const int iz = i0[2] + (int)(i / ((int64_t)n[0] * n[1]));
            const double xx = box.lo[0] + (ix + 0.5) * box.vs[0] - p[0];
            const double yy = box.lo[1] + (iy + 0.5) * box.vs[1] - p[1];
            const double zz = box.lo[2] + (iz + 0.5) * box.vs[2] - p[2];
            const double d2 = xx * xx + yy * yy + zz * zz;
            if (!(d2 <= r2)) continue;
            const double v = log1p(-o * exp(-0.5 * d2 / (sig * sig)));
            const long long q = llrint(v * OCC_SCALE);
            atomicAdd(acc + ((size_t)iz * G + iy) * G + ix, (unsigned long long)q);
        }
    }
}

// V = 1 - exp(sum)
__global__ __launch_bounds__(BLOCK) void k_rc_finish(const unsigned long long *__restrict__ acc, size_t n,
                                                     float *__restrict__ occ)
{
    const size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const double s = (double)(long long)acc[i] / OCC_SCALE;
    occ[i] = (float)(-expm1(s));
}

// coefficients K x L x C (component index order) -> walk order
__global__ __launch_bounds__(BLOCK) void k_rc_coef_perm(const float2 *__restrict__ in, int64_t K, int L, int C,
                                                        const int *__restrict__ walk, float2 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t n = K * L * C;
    if (i >= n) return;
    const int c = (int)(i % C);
    const int64_t kw = i / C;
    const int w = (int)(kw % L);
    const int64_t k = kw / L;
    out[i] = in[(k * L + walk[w]) * C + c];
}

// ---------------------------------------------------------------------------
// receiver terms

// gam[j][u] = sum_i W1[u][2i] sin(w_i . r_j) + W1[u][2i + 1] cos(w_i . r_j)
// (eq. rx_enc into the global MLP's first layer); the encoding in FP64, since
// its arguments reach hundreds of radians
__global__ __launch_bounds__(BLOCK) void k_rxcond_gamma(const float *__restrict__ wfreq, const float *__restrict__ gw1,
                                                        int F, int gin, const float *__restrict__ rx, int N,
                                                        float *__restrict__ gam)
{
#pragma clang fp contract(off)
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= N * RC_H) return;
    const int j = idx / RC_H, u = idx % RC_H;
    const double r0 = rx[3 * j], r1 = rx[3 * j + 1], r2 = rx[3 * j + 2];
    const float *row = gw1 + (size_t)u * gin;
    double acc = 0.0;
    for (int i = 0; i < 3 * F; i++) {
        const double a = (double)wfreq[3 * i] * r0 + (double)wfreq[3 * i + 1] * r1 + (double)wfreq[3 * i + 2] * r2;
        double sn, cs;
        sincos(a, &sn, &cs);
        acc += (double)row[2 * i] * sn;
        acc += (double)row[2 * i + 1] * cs;
    }
    gam[idx] = (float)acc;
}

// The global MLP (eq. film) per (receiver j, walk position w), one wave each:
// h1 = relu(gam_j + comp_w) (comp_w = b1 + W1 [deg/m, ord/m; e_l]), h2 =
// relu(W2 h1 + b2), out = W3 h2 + b3; rab[j][w][c] = (1 + alpha, beta).
// Lane u holds hidden unit u; W2 and W3 are staged transposed in LDS.
__global__ __launch_bounds__(BLOCK) void k_rxcond_global(const float *__restrict__ gam,
                                                         const float *__restrict__ comp,
                                                         const float *__restrict__ gw2, const float *__restrict__ gb2,
                                                         const float *__restrict__ gw3, const float *__restrict__ gb3,
                                                         int N, int L, int C, float *__restrict__ rab)
{
    extern __shared__ float s_dyn[];
    float *s_w2t = s_dyn;                 // [v][u] = W2[u][v]
    float *s_w3t = s_dyn + RC_H * RC_H;   // [u][o] = W3[o][u]
    const int nout = 4 * C;
    for (int i = threadIdx.x; i < RC_H * RC_H; i += BLOCK) s_w2t[(i % RC_H) * RC_H + i / RC_H] = gw2[i];
    for (int i = threadIdx.x; i < nout * RC_H; i += BLOCK) s_w3t[(i % RC_H) * nout + i / RC_H] = gw3[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t total = (int64_t)N * L;
    const float b2 = gb2[lane];
    for (int64_t it = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); it < total;
         it += (int64_t)gridDim.x * (BLOCK / 64)) {
        const int j = (int)(it / L), w = (int)(it % L);
        const float h1 = fmaxf(gam[(size_t)j * RC_H + lane] + comp[(size_t)w * RC_H + lane], 0.f);
        float a = b2;
        for (int v = 0; v < RC_H; v++) a = fmaf(s_w2t[v * RC_H + lane], __shfl(h1, v), a);
        const float h2 = fmaxf(a, 0.f);
        float *dst = rab + (size_t)it * nout;
        for (int o0 = 0; o0 < nout; o0 += 64) {
            const int o = o0 + lane;
            const int oc = min(o, nout - 1);
            float y = gb3[oc];
            for (int u = 0; u < RC_H; u++) y = fmaf(s_w3t[u * nout + oc], __shfl(h2, u), y);
            if (o < nout) dst[o] = (o & 3) == 0 ? 1.f + y : y;
        }
    }
}

// ---------------------------------------------------------------------------
// per-pair kernels over MLP work items (view, s0, first receiver, receivers |
// valid positions << 8); one wave per item, lanes l and l + 32 share the
// pair of sorted position s0 + l % 32

// Local branch (eqs. transmittance, local): probes, then the local MLP.
// Layer 1 by lane half h for hidden units 2t + h; layer 2 on FP32 MFMA with
// A = W2 (w2t[(32 b + t) 64 + lane] = W2[32 b + lane % 32][2 t + lane / 32])
// and B = layer-1 outputs, so accumulator register r of block b in lane half
// h is hidden unit 32 b + 8 (r / 4) + 4 h + r % 4 of the lane's pair; layer 3
// as per-lane dot products over those 32 units plus one exchange.
__global__ __launch_bounds__(BLOCK) void k_rxcond_local(
    const float *__restrict__ soa, int64_t K, const float *__restrict__ rxpos, const uint32_t *__restrict__ order,
    const int4 *__restrict__ items, int nitems, const int *__restrict__ nlive, int64_t Kp,
    const float *__restrict__ occ, int G, RcBox box, const double *__restrict__ tprobe, int S,
    const float *__restrict__ lw1, const float *__restrict__ lb1, const float *__restrict__ w2t,
    const float *__restrict__ lb2, const float *__restrict__ lw3, const float *__restrict__ lb3, int C, int rpu,
    float4 *__restrict__ rloc)
{
#pragma clang fp contract(off)
    if (nlive) nitems = min(nitems, *nlive);
    __shared__ float s_w1[RC_H * 7];
    __shared__ float s_w2[2 * 32 * 64];
    __shared__ float s_b2[RC_H];
    __shared__ double s_t[64];
    extern __shared__ float s_dyn[];
    const int nout = 4 * C;
    float *s_w3 = s_dyn;            // [o][h][32]: W3[o][unit of (h, slot)]
    float *s_b3 = s_dyn + nout * RC_H;
    for (int i = threadIdx.x; i < RC_H * 6; i += BLOCK) s_w1[(i / 6) * 7 + i % 6] = lw1[i];
    for (int i = threadIdx.x; i < RC_H; i += BLOCK) {
        s_w1[i * 7 + 6] = lb1[i];
        s_b2[i] = lb2[i];
    }
    for (int i = threadIdx.x; i < 2 * 32 * 64; i += BLOCK) s_w2[i] = w2t[i];
    for (int i = threadIdx.x; i < S; i += BLOCK) s_t[i] = tprobe[i];
    for (int i = threadIdx.x; i < nout * RC_H; i += BLOCK) {
        const int o = i / RC_H, rem = i % RC_H, hh = rem / 32, slot = rem % 32;
        const int b = slot / 16, r = slot % 16;
        s_w3[i] = lw3[(size_t)o * RC_H + 32 * b + 8 * (r >> 2) + 4 * hh + (r & 3)];
    }
    for (int i = threadIdx.x; i < nout; i += BLOCK) s_b3[i] = lb3[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, h = lane >> 5, pl = lane & 31;
    const float invS = 1.f / (float)S;
    // one unit = (work item, one of its receivers): rpu units per item
    const int nunits = nitems * rpu;
    for (int u = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); u < nunits; u += gridDim.x * (BLOCK / 64)) {
        const int item = u / rpu, jj = u - item * rpu;
        const int4 it = items[item];
        const int view = it.x, s0 = it.y, j0 = it.z, nj = it.w & 255, nvalid = it.w >> 8;
        if (jj >= nj) continue;
        const bool valid = pl < nvalid;
        const int64_t s = s0 + pl;
        const int64_t k = min((int64_t)order[(size_t)view * Kp + (valid ? s : s0)], K - 1);
        const float px = soa[k], py = soa[K + k], pz = soa[2 * K + k];
        const double pd[3] = {(double)px, (double)py, (double)pz};
        {
            const int j = j0 + jj;
            const float rxx = rxpos[3 * j], rxy = rxpos[3 * j + 1], rxz = rxpos[3 * j + 2];
            const double rd[3] = {(double)rxx, (double)rxy, (double)rxz};
            // probes q_s = p + t_s (r - p): this half takes s = h, h + 2, ...
            float Th = 1.f, Sh = 0.f;
            for (int si = h; si < S; si += 2) {
                const double t = s_t[si];
                bool inside = true;
                int id[3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const double q = pd[a] + t * (rd[a] - pd[a]);
                    const double uu = (q - box.lo[a]) * box.inv[a];
                    const double fl = floor(uu);
                    inside = inside && fl >= 0.0 && fl <= (double)(G - 1);
                    id[a] = inside ? (int)fl : 0;
                }
                const float vv = inside ? occ[((size_t)id[2] * G + id[1]) * G + id[0]] : 0.f;
                Th *= 1.f - vv;
                Sh += vv;
            }
            const float T = Th * __shfl_xor(Th, 32);
            const float rho = (Sh + __shfl_xor(Sh, 32)) * invS;
            const float vx = rxx - px, vy = rxy - py, vz = rxz - pz;
            const float d = sqrtf(vx * vx + vy * vy + vz * vz);
            const float id_ = d > 0.f ? 1.f / d : 0.f;
            const float f[6] = {vx * id_, vy * id_, vz * id_, d, T, rho};
            // layer 1: hidden units 2t + h
            float h1[32];
#pragma unroll
            for (int t = 0; t < 32; t++) {
                const float *w = s_w1 + (2 * t + h) * 7;
                float a = w[6];
#pragma unroll
                for (int i = 0; i < 6; i++) a = fmaf(w[i], f[i], a);
                h1[t] = fmaxf(a, 0.f);
            }
            // layer 2 (64 x 64) on FP32 MFMA
            floatx16 acc0, acc1;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int m = 8 * (r >> 2) + 4 * h + (r & 3);
                acc0[r] = s_b2[m];
                acc1[r] = s_b2[32 + m];
            }
#pragma unroll
            for (int t = 0; t < 32; t++) {
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(s_w2[t * 64 + lane], h1[t], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(s_w2[(32 + t) * 64 + lane], h1[t], acc1, 0, 0, 0);
            }
            float h2[32];
#pragma unroll
            for (int r = 0; r < 16; r++) {
                h2[r] = fmaxf(acc0[r], 0.f);
                h2[16 + r] = fmaxf(acc1[r], 0.f);
            }
            // layer 3, one channel (4 outputs) at a time
            for (int c = 0; c < C; c++) {
                float y[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const float *w = s_w3 + ((4 * c + e) * 2 + h) * 32;
                    float a = 0.f;
#pragma unroll
                    for (int q = 0; q < 32; q++) a = fmaf(w[q], h2[q], a);
                    y[e] = a + __shfl_xor(a, 32) + s_b3[4 * c + e];
                }
                if (valid && (c & 1) == h)
                    rloc[((size_t)j * Kp + s) * C + c] = make_float4(1.f + y[0], y[1], y[2], y[3]);
            }
        }
    }
}

// Basis reduction (App. E.2; Alg. 1 eval_fle) and the two modulations.  For
// each receiver and channel pass the lane walks its half of the components:
// X_c += ((1 + alpha) phi + beta) B_l over them, and the basis sum SB; the
// halves are added, then s_c = (1 + alpha') X_c + beta' SB (eq.
// combined_local summed against the basis).
template <int KIND>
__global__ __launch_bounds__(BLOCK) void k_rxcond_eval(
    const float *__restrict__ soa, int64_t K, const float *__restrict__ centres, const uint32_t *__restrict__ order,
    const int4 *__restrict__ items, int nitems, const int *__restrict__ nlive, int64_t Kp,
    const float2 *__restrict__ coef, const float4 *__restrict__ rab, const float4 *__restrict__ rloc,
    const float4 *__restrict__ ctab, int lmax, int L, int n0, int C, int rpu, float2 *__restrict__ rad)
{
    if (nlive) nitems = min(nitems, *nlive);
    __shared__ float4 s_ct[RC_TAB * RC_TAB];
    for (int i = threadIdx.x; i < RC_TAB * RC_TAB; i += BLOCK) s_ct[i] = ctab[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, h = lane >> 5, pl = lane & 31;
    const float SQ2 = 1.41421356237309515f;
    const int nunits = nitems * rpu;
    for (int u = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); u < nunits; u += gridDim.x * (BLOCK / 64)) {
        const int item = u / rpu, ju = u - item * rpu;
        const int4 it = items[item];
        const int view = it.x, s0 = it.y, j0 = it.z, nj = it.w & 255, nvalid = it.w >> 8;
        if (ju >= nj) continue;
        const bool valid = pl < nvalid;
        const int64_t s = s0 + pl;
        const int64_t k = min((int64_t)order[(size_t)view * Kp + (valid ? s : s0)], K - 1);
        const float dx = soa[k] - centres[3 * view];
        const float dy = soa[K + k] - centres[3 * view + 1];
        const float dz = soa[2 * K + k] - centres[3 * view + 2];
        const float rh2 = dx * dx + dy * dy;
        const float rh = sqrtf(rh2), rr = sqrtf(rh2 + dz * dz);
        const float ir = rr > 0.f ? 1.f / rr : 0.f;
        const float x = dz * ir, sn = rh * ir;            // cos and sin of the polar angle
        const float cp = rh > 0.f ? dx / rh : 1.f;         // cos and sin of the azimuth
        const float sp = rh > 0.f ? dy / rh : 0.f;
        const float c2 = cp * cp - sp * sp, s2 = 2.f * cp * sp;
        const float2 *crow = coef + (size_t)k * L * C;
        {
            const int j = j0 + ju;
            const float4 *arow = rab + (size_t)j * L * C;
            for (int c0 = 0; c0 < C; c0 += RC_CH_PASS) {
                const int nc = min(RC_CH_PASS, C - c0);
                float xr[RC_CH_PASS], xi[RC_CH_PASS];
#pragma unroll
                for (int q = 0; q < RC_CH_PASS; q++) xr[q] = xi[q] = 0.f;
                float br = 0.f, bi = 0.f;
                int w = h ? n0 : 0;
                // one component: basis value (Br, Bi) at walk position w
                auto acc_comp = [&](float Br, float Bi) {
                    br += Br;
                    bi += Bi;
                    const float2 *cf = crow + (size_t)w * C + c0;
                    const float4 *ab = arow + (size_t)w * C + c0;
#pragma unroll
                    for (int q = 0; q < RC_CH_PASS; q++) {
                        if (q < nc) {
                            const float2 f = cf[q];
                            const float4 a = ab[q];
                            const float tr = fmaf(a.x, f.x, fmaf(-a.y, f.y, a.z));
                            const float ti = fmaf(a.x, f.y, fmaf(a.y, f.x, a.w));
                            if (KIND == RXGS_BASIS_FLE) {
                                xr[q] = fmaf(tr, Br, fmaf(-ti, Bi, xr[q]));
                                xi[q] = fmaf(tr, Bi, fmaf(ti, Br, xi[q]));
                            } else {
                                xr[q] = fmaf(tr, Br, xr[q]);
                                xi[q] = fmaf(ti, Br, xi[q]);
                            }
                        }
                    }
                    w++;
                };
                float pmm = h ? sn : 1.f;                  // P_m^m at m = h
                float cm = h ? cp : 1.f, sm = h ? sp : 0.f; // cos(m ph), sin(m ph)
                for (int m = h; m <= lmax; m += 2) {
                    float p2 = 0.f, p1 = 0.f;
                    for (int l = m; l <= lmax; l++) {
                        const float4 ct = s_ct[l * RC_TAB + m];   // (N_lm, a_lm, b_lm, -)
                        float P;
                        if (l == m) P = pmm;
                        else if (l == m + 1) P = x * (float)(2 * m + 1) * pmm;
                        else P = ct.y * x * p1 - ct.z * p2;
                        p2 = p1;
                        p1 = P;
                        const float np = ct.x * P;
                        if (m == 0) {
                            acc_comp(np, 0.f);
                        } else if (KIND == RXGS_BASIS_FLE) {
                            acc_comp(np * cm, np * sm);
                            acc_comp(np * cm, -np * sm);
                        } else {
                            acc_comp(SQ2 * np * cm, 0.f);
                            acc_comp(SQ2 * np * sm, 0.f);
                        }
                    }
                    pmm *= (float)((2 * m + 1) * (2 * m + 3)) * sn * sn;
                    const float cn = cm * c2 - sm * s2;
                    sm = sm * c2 + cm * s2;
                    cm = cn;
                }
                br += __shfl_xor(br, 32);
                bi += __shfl_xor(bi, 32);
#pragma unroll
                for (int q = 0; q < RC_CH_PASS; q++) {
                    if (q < nc) {
                        xr[q] += __shfl_xor(xr[q], 32);
                        xi[q] += __shfl_xor(xi[q], 32);
                    }
                }
#pragma unroll
                for (int q = 0; q < RC_CH_PASS; q++) {
                    if (q < nc && valid && (q & 1) == h) {
                        const int c = c0 + q;
                        const float4 lm = rloc[((size_t)j * Kp + s) * C + c];
                        const float sr = lm.x * xr[q] - lm.y * xi[q] + lm.z * br - lm.w * bi;
                        const float si = lm.x * xi[q] + lm.y * xr[q] + lm.z * bi + lm.w * br;
                        rad[((size_t)j * C + c) * Kp + s] = make_float2(sr, si);
                    }
                }
            }
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

void release_rxcond(RxCond &m)
{
    DevBuf *bufs[] = {&m.coef, &m.params, &m.comp, &m.walk, &m.ctab, &m.tprobe, &m.occ, &m.w2t};
    for (DevBuf *b : bufs) release(*b);
    m.valid = false;
}

RcOffsets rc_offsets(int L, int C, int F)
{
    RcOffsets o;
    const size_t gin = (size_t)6 * F + 2 + RXGS_RXCOND_EMB;
    o.w = 0;
    o.e = o.w + (size_t)9 * F;
    o.g1 = o.e + (size_t)L * RXGS_RXCOND_EMB;
    o.gb1 = o.g1 + RC_H * gin;
    o.g2 = o.gb1 + RC_H;
    o.gb2 = o.g2 + RC_H * RC_H;
    o.g3 = o.gb2 + RC_H;
    o.gb3 = o.g3 + (size_t)4 * C * RC_H;
    o.l1 = o.gb3 + (size_t)4 * C;
    o.lb1 = o.l1 + RC_H * 6;
    o.l2 = o.lb1 + RC_H;
    o.lb2 = o.l2 + RC_H * RC_H;
    o.l3 = o.lb2 + RC_H;
    o.lb3 = o.l3 + (size_t)4 * C * RC_H;
    o.total = o.lb3 + (size_t)4 * C;
    return o;
}

float rc_key_value(unsigned key)
{
    const unsigned b = (key & 0x80000000u) ? (key & 0x7FFFFFFFu) : ~key;
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

hipError_t launch_rc_bounds(const Scene &sc, unsigned *keys, hipStream_t st)
{
    if (sc.K == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((sc.K + BLOCK - 1) / BLOCK, 1024);
    hipLaunchKernelGGL(k_rc_bounds, dim3(blocks), dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K, keys);
    return hipGetLastError();
}

static RcBox rc_box(const RxCond &m)
{
    RcBox b;
    for (int a = 0; a < 3; a++) {
        b.lo[a] = m.lo[a];
        b.inv[a] = m.inv[a];
        b.vs[a] = m.vs[a];
    }
    return b;
}

hipError_t launch_rc_splat(const Scene &sc, const RxCond &m, unsigned long long *acc, hipStream_t st)
{
    if (sc.K == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((sc.K + 3) / 4, 8192);
    hipLaunchKernelGGL(k_rc_splat, dim3(blocks), dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K, m.G, rc_box(m), acc);
    return hipGetLastError();
}

hipError_t launch_rc_finish(const RxCond &m, const unsigned long long *acc, hipStream_t st)
{
    const size_t n = (size_t)m.G * m.G * m.G;
    hipLaunchKernelGGL(k_rc_finish, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, acc, n,
                       m.occ.as<float>());
    return hipGetLastError();
}

hipError_t launch_rc_coef_perm(const float *src, int64_t K, const RxCond &m, hipStream_t st)
{
    const int64_t n = K * m.L * m.C;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rc_coef_perm, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st,
                       reinterpret_cast<const float2 *>(src), K, m.L, m.C, m.walk.as<int>(), m.coef.as<float2>());
    return hipGetLastError();
}

// receiver terms: the encoding into layer 1, then the global MLP per
// (receiver, component); ws.rxpos_p holds the Nrx receivers
hipError_t launch_rxcond_receivers(const RxCond &m, Workspace &ws, hipStream_t st)
{
    const int N = ws.Nrx;
    if (N == 0) return hipSuccess;
    if (ws.rgam.cap < (size_t)N * RC_H * 4 || ws.rab.cap < (size_t)N * m.L * m.C * 16) return hipErrorInvalidValue;
    const float *P = m.params.as<float>();
    const int gin = 6 * m.F + 2 + RXGS_RXCOND_EMB;
    hipLaunchKernelGGL(k_rxcond_gamma, dim3((unsigned)((N * RC_H + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st,
                       P + m.off.w, P + m.off.g1, m.F, gin, ws.rxpos_p, N, ws.rgam.as<float>());
    const int64_t waves = (int64_t)N * m.L;
    const unsigned blocks = (unsigned)std::min<int64_t>((waves + 3) / 4, 4096);
    const size_t lds = (size_t)(RC_H * RC_H + 4 * m.C * RC_H) * 4;
    hipLaunchKernelGGL(k_rxcond_global, dim3(blocks), dim3(BLOCK), lds, st, ws.rgam.as<float>(), m.comp.as<float>(),
                       P + m.off.g2, P + m.off.gb2, P + m.off.g3, P + m.off.gb3, N, m.L, m.C, ws.rab.as<float>());
    return hipGetLastError();
}

// per-pair work over the MLP work items: the prefix's (or all), the live ones
// (lazy TX), or those past the prefix of the views that need them
hipError_t launch_rxcond_pairs(const Scene &sc, const RxCond &m, Workspace &ws, hipStream_t st, bool far)
{
    const int4 *items = far ? ws.items_far.as<int4>() : ws.lazy ? ws.items_live.as<int4>() : ws.items.as<int4>();
    const int *nlive = far ? far_count(ws) : ws.lazy ? live_count(ws) : nullptr;
    const int nmax = far ? ws.n_items_far : ws.n_items;
    if (nmax <= 0) return hipSuccess;
    // a wave per (item, receiver): items carry up to MLP_RG receivers of a view
    const int rpu = std::max(1, std::min(MLP_RG, ws.rx_max));
    const unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)nmax * rpu + 3) / 4, 256 * 8);
    const float *P = m.params.as<float>();
    RcBox box = rc_box(m);
    const size_t lds = (size_t)(4 * m.C * RC_H + 4 * m.C) * 4;
    hipLaunchKernelGGL(k_rxcond_local, dim3(blocks), dim3(BLOCK), lds, st, sc.soa.as<float>(), sc.K, ws.rxpos_p,
                       ws.vorder.as<uint32_t>(), items, nmax, nlive, ws.Kp, m.occ.as<float>(), m.G, box,
                       m.tprobe.as<double>(), m.S, P + m.off.l1, P + m.off.lb1, m.w2t.as<float>(), P + m.off.lb2,
                       P + m.off.l3, P + m.off.lb3, m.C, rpu, ws.rloc.as<float4>());
    if (m.kind == RXGS_BASIS_FLE)
        hipLaunchKernelGGL(k_rxcond_eval<RXGS_BASIS_FLE>, dim3(blocks), dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K,
                           ws.centres_p, ws.vorder.as<uint32_t>(), items, nmax, nlive, ws.Kp, m.coef.as<float2>(),
                           ws.rab.as<float4>(), ws.rloc.as<float4>(), m.ctab.as<float4>(), m.lmax, m.L, m.n0, m.C,
                           rpu, ws.rad.as<float2>());
    else
        hipLaunchKernelGGL(k_rxcond_eval<RXGS_BASIS_SH>, dim3(blocks), dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K,
                           ws.centres_p, ws.vorder.as<uint32_t>(), items, nmax, nlive, ws.Kp, m.coef.as<float2>(),
                           ws.rab.as<float4>(), ws.rloc.as<float4>(), m.ctab.as<float4>(), m.lmax, m.L, m.n0, m.C,
                           rpu, ws.rad.as<float2>());
    return hipGetLastError();
}

}  // namespace rxgs
