// Forward kernels of librxgs for gfx950 (CDNA4, wave64).
//
// Pipeline of one render (Alg. 1 of RxGS, arXiv 2605.24290, with the view
// index added to the sort key):
//   k_project      stage 1: per (view, Gaussian) projection onto the angular
//                  grid, FP32 depth key, conservative tile count.   [HBM]
//   radix sort     stage 1: per-view stable sort of the depth keys (one
//                  segment per view), 4 passes of 8 bits (sort.hip). [HBM]
//   k_gather       records into depth order, tile counts in depth order.
//   scan + k_emit  one (local tile, sorted position) pair per covered tile,
//                  emitted in depth order into the view's segment.  [HBM]
//   radix sort     stable 8-bit sort of each view's pairs by tile, so each
//                  tile's list stays in depth order.                [HBM]
//   k_ranges_hist  [start, end) of each tile's list.
//   k_mlp_*        stage 2: receiver term and Gaussian term of the MLP's first
//                  layer, then the per-(receiver, Gaussian) layers on split
//                  FP16 MFMA.                                       [MFMA]
//   k_blend_fwd    stage 3: per (tile, receiver chunk) front-to-back
//                  compositing from LDS-staged batches.             [VALU]
//   k_reduce_out   per-receiver power and coherent sum, fixed order.
#include "device_common.h"

#include <cmath>

namespace rxgs {

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ float wave_sum_f32(float x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// FP32 squared distance, each product and sum rounded on its own (no FMA)
__device__ __forceinline__ float depth_key(float dx, float dy, float dz)
{
#pragma clang fp contract(off)
    const float xx = dx * dx;
    const float yy = dy * dy;
    const float zz = dz * dz;
    return (xx + yy) + zz;
}

// ----------------------------------------------------------------------------
// tile coverage of one record, FP32 rules (rows clamped to the grid, columns
// modulo W; a box spanning nearly the full circle takes every tile column)
__device__ __forceinline__ int tile_rows(float v, float rvp, int H, int &ty0, int &ty1)
{
    float lo = fmaxf(__fsub_rn(v, rvp), 0.0f);
    float hi = fminf(__fadd_rn(v, rvp), (float)(H - 1));
    int i0 = (int)ceilf(lo), i1 = (int)floorf(hi);
    if (i0 > i1) return 0;
    ty0 = i0 / TILE;
    ty1 = i1 / TILE;
    return ty1 - ty0 + 1;
}

__device__ __forceinline__ int tile_cols(float u, float rup, int W, int tiles_x, int &a0, int &a1, int &b0,
                                         int &b1)
{
    b0 = 0;
    b1 = -1;
    if (rup >= 0.5f * (float)(W - TILE - 2)) {
        a0 = 0;
        a1 = tiles_x - 1;
        return tiles_x;
    }
    int c0 = (int)ceilf(__fsub_rn(u, rup)), c1 = (int)floorf(__fadd_rn(u, rup));
    if (c0 > c1) return 0;
    int m = ((c0 % W) + W) % W;
    int e = m + (c1 - c0);
    a0 = m / TILE;
    if (e < W) {
        a1 = e / TILE;
    } else {
        a1 = (W - 1) / TILE;
        b1 = (e - W) / TILE;
    }
    return (a1 - a0 + 1) + (b1 - b0 + 1);
}

// ----------------------------------------------------------------------------
// Stage 1: projection.  One thread per Gaussian (coalesced SoA loads), looping
// over a chunk of views.  Geometry in FP64 (exact differences of the FP32
// inputs), stored as FP32.  The depth key is the FP32 squared distance
// computed with rounded, unfused operations.
__global__ __launch_bounds__(BLOCK) void k_project(
    const float *__restrict__ soa, int64_t K, int64_t Kp, const float *__restrict__ centres, int V,
    int vchunk, DevGrid g, float4 *__restrict__ rec, float4 *__restrict__ ext, uint32_t *__restrict__ rawkey,
    float *__restrict__ opac, uint32_t *__restrict__ ntl, uint32_t *__restrict__ skey,
    uint32_t *__restrict__ sval, unsigned long long *__restrict__ counters)
{
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int v0 = blockIdx.y * vchunk;
    const int v1 = min(V, v0 + vchunk);
    const bool real = k < K;
    __shared__ uint32_t s_cnt[4][2];
    const int lane = threadIdx.x & 63;
    float px = 0.f, py = 0.f, pz = 0.f, o32 = 0.f;
    double qmax = 0.0, lo2 = 0.0;
    double S00 = 0, S01 = 0, S02 = 0, S11 = 0, S12 = 0, S22 = 0;
    if (real) {
        px = soa[k];
        py = soa[K + k];
        pz = soa[2 * K + k];
        const double s0 = exp(2.0 * (double)soa[3 * K + k]);
        const double s1 = exp(2.0 * (double)soa[4 * K + k]);
        const double s2 = exp(2.0 * (double)soa[5 * K + k]);
        double qw = soa[6 * K + k], qx = soa[7 * K + k], qy = soa[8 * K + k], qz = soa[9 * K + k];
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        const double R00 = 1.0 - 2.0 * (qy * qy + qz * qz), R01 = 2.0 * (qx * qy - qw * qz),
                     R02 = 2.0 * (qx * qz + qw * qy);
        const double R10 = 2.0 * (qx * qy + qw * qz), R11 = 1.0 - 2.0 * (qx * qx + qz * qz),
                     R12 = 2.0 * (qy * qz - qw * qx);
        const double R20 = 2.0 * (qx * qz - qw * qy), R21 = 2.0 * (qy * qz + qw * qx),
                     R22 = 1.0 - 2.0 * (qx * qx + qy * qy);
        S00 = R00 * R00 * s0 + R01 * R01 * s1 + R02 * R02 * s2;
        S01 = R00 * R10 * s0 + R01 * R11 * s1 + R02 * R12 * s2;
        S02 = R00 * R20 * s0 + R01 * R21 * s1 + R02 * R22 * s2;
        S11 = R10 * R10 * s0 + R11 * R11 * s1 + R12 * R12 * s2;
        S12 = R10 * R20 * s0 + R11 * R21 * s1 + R12 * R22 * s2;
        S22 = R20 * R20 * s0 + R21 * R21 * s1 + R22 * R22 * s2;
        o32 = (float)(1.0 / (1.0 + exp(-(double)soa[10 * K + k])));
        if (o32 >= ALPHA_MIN) {
            qmax = 2.0 * log((double)o32 / (double)ALPHA_MIN);
            lo2 = log2((double)o32);
        }
    }
    for (int v = v0; v < v1; v++) {
        const size_t i = (size_t)v * Kp + k;
        uint32_t key = 0xFFFFFFFFu, kb = 0xFFFFFFFFu, nt = 0;
        float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
        bool vis = false;
        if (real) {
            const float cx = centres[3 * v], cy = centres[3 * v + 1], cz = centres[3 * v + 2];
            const float dxf = __fsub_rn(px, cx), dyf = __fsub_rn(py, cy), dzf = __fsub_rn(pz, cz);
            const float kf = depth_key(dxf, dyf, dzf);
            kb = __float_as_uint(kf);
            if (!(kf < NEAR2)) {
                const double dx = (double)px - (double)cx, dy = (double)py - (double)cy,
                             dz = (double)pz - (double)cz;
                double h = sqrt(dx * dx + dy * dy);
                if (!(h >= H_MIN)) h = H_MIN;
                double az = atan2(dy, dx);
                if (az < 0.0) az += 2.0 * M_PI;
                const double el = atan2(dz, h);
                const double u = az * g.idaz - 0.5;
                const double vv = (el - g.el0) * g.idel - 0.5;
                const double hh = h * h, rh2 = hh + dz * dz;
                const double ihh = g.idaz / hh;               // 1 / (h^2 daz)
                const double irh = g.idel / (rh2 * h);        // 1 / (rho^2 h del)
                const double mu0 = -dy * ihh, mu1 = dx * ihh;
                const double mv0 = -dx * dz * irh, mv1 = -dy * dz * irh, mv2 = hh * irh;
                const double Smv0 = S00 * mv0 + S01 * mv1 + S02 * mv2;
                const double Smv1 = S01 * mv0 + S11 * mv1 + S12 * mv2;
                const double Smv2 = S02 * mv0 + S12 * mv1 + S22 * mv2;
                const double A = S00 * mu0 * mu0 + 2.0 * S01 * mu0 * mu1 + S11 * mu1 * mu1 + DILATE;
                const double B = mu0 * Smv0 + mu1 * Smv1;
                const double Cc = mv0 * Smv0 + mv1 * Smv1 + mv2 * Smv2 + DILATE;
                const float u32 = (float)u, v32 = (float)vv;
                e = make_float4(u32, v32, 0.f, 0.f);
                if (o32 >= ALPHA_MIN) {
                    const float rup = (float)(sqrt(qmax * A) * (1.0 + PAD_REL) + PAD_ABS);
                    const float rvp = (float)(sqrt(qmax * Cc) * (1.0 + PAD_REL) + PAD_ABS);
                    e.z = rup;
                    e.w = rvp;
                    int ty0, ty1, a0, a1, b0, b1;
                    const int nr = tile_rows(v32, rvp, g.H, ty0, ty1);
                    const int nc = nr ? tile_cols(u32, rup, g.W, g.tiles_x, a0, a1, b0, b1) : 0;
                    nt = (uint32_t)(nr * nc);
                }
                vis = nt > 0;
                if (vis) {
                    const double idet = 1.0 / (A * Cc - B * B);
                    const double ca = Cc * idet, cb = -B * idet, cc = A * idet;
                    const double uf = floor(u), vf = floor(vv);
                    constexpr double L2E = 1.4426950408889634;
                    rec[2 * i] = make_float4((float)uf, (float)(u - uf), (float)vf, (float)(vv - vf));
                    rec[2 * i + 1] = make_float4((float)(-0.5 * L2E * ca), (float)(-L2E * cb),
                                                 (float)(-0.5 * L2E * cc), (float)lo2);
                    key = kb;
                }
            }
        }
        ext[i] = e;
        rawkey[i] = kb;
        opac[i] = o32;
        ntl[i] = nt;
        skey[i] = key;
        sval[i] = (uint32_t)k;
        const uint64_t bal = __ballot(vis);
        const uint32_t tsum = wave_sum_u32(nt);
        if (lane == 0) {
            s_cnt[threadIdx.x >> 6][0] = (uint32_t)__popcll(bal);
            s_cnt[threadIdx.x >> 6][1] = tsum;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t nv = s_cnt[0][0] + s_cnt[1][0] + s_cnt[2][0] + s_cnt[3][0];
            const uint32_t nd = s_cnt[0][1] + s_cnt[1][1] + s_cnt[2][1] + s_cnt[3][1];
            if (nv) atomicAdd(&counters[2 * (size_t)v], (unsigned long long)nv);
            if (nd) atomicAdd(&counters[2 * (size_t)v + 1], (unsigned long long)nd);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// fills
__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t value, size_t n)
{
    size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * BLOCK;
    for (; i < n; i += stride) p[i] = value;
}

// ----------------------------------------------------------------------------
// exclusive scan of u32 (three kernels: block sums, scan of block sums,
// block-local scan plus offset); blocks of 4096, 16 consecutive items per thread
__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const uint32_t *__restrict__ in, uint32_t n,
                                                       uint32_t *__restrict__ bsum)
{
    __shared__ uint32_t s_w[4];
    const size_t base = (size_t)blockIdx.x * SORT_TILE + (size_t)threadIdx.x * SORT_ITEMS;
    uint32_t s = 0;
    for (int i = 0; i < SORT_ITEMS; i++)
        if (base + i < n) s += in[base + i];
    s = wave_sum_u32(s);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// single workgroup: exclusive scan of nb values (in may equal out)
__global__ __launch_bounds__(BLOCK) void k_scan_top(const uint32_t *in, uint32_t *out, uint32_t nb)
{
    __shared__ uint32_t s_w[4];
    uint32_t carry = 0;
    for (uint32_t c = 0; c < nb; c += SORT_TILE) {
        const uint32_t base = c + threadIdx.x * SORT_ITEMS;
        uint32_t loc[SORT_ITEMS];
        uint32_t s = 0;
        for (int i = 0; i < SORT_ITEMS; i++) {
            loc[i] = (base + i < nb) ? in[base + i] : 0u;
            s += loc[i];
        }
        uint32_t tot;
        uint32_t pre = block_exclusive_scan(s, tot, s_w) + carry;
        for (int i = 0; i < SORT_ITEMS; i++) {
            if (base + i < nb) out[base + i] = pre;
            pre += loc[i];
        }
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLOCK) void k_scan_down(const uint32_t *__restrict__ in, uint32_t n,
                                                     const uint32_t *__restrict__ bsum,
                                                     uint32_t *__restrict__ out)
{
    __shared__ uint32_t s_w[4];
    const size_t base = (size_t)blockIdx.x * SORT_TILE + (size_t)threadIdx.x * SORT_ITEMS;
    uint32_t loc[SORT_ITEMS];
    uint32_t s = 0;
    for (int i = 0; i < SORT_ITEMS; i++) {
        loc[i] = (base + i < n) ? in[base + i] : 0u;
        s += loc[i];
    }
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, tot, s_w) + bsum[blockIdx.x];
    for (int i = 0; i < SORT_ITEMS; i++) {
        if (base + i < n) out[base + i] = pre;
        pre += loc[i];
    }
}

// records into depth order; tile counts in depth order
__global__ __launch_bounds__(BLOCK) void k_gather(const float4 *__restrict__ rec, const uint32_t *__restrict__ ntl,
                                                  const uint32_t *__restrict__ order,
                                                  const unsigned long long *__restrict__ counters, int64_t Kp,
                                                  int64_t total, float4 *__restrict__ srec,
                                                  uint32_t *__restrict__ ntl_s)
{
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= total) return;
    const int64_t v = p / Kp, s = p - v * Kp;
    if (s < (int64_t)counters[2 * (size_t)v]) {
        const size_t i = (size_t)v * Kp + min((int64_t)order[p], Kp - 1);
        srec[2 * p] = rec[2 * i];
        srec[2 * p + 1] = rec[2 * i + 1];
        ntl_s[p] = ntl[i];
    } else {
        ntl_s[p] = 0;
    }
}

// One pair (local tile id, sorted position) per covered tile, in depth order
// within the view, into the view's segment of the pair arrays (segments start
// at multiples of 4096 so the pair sort can treat each view on its own; the
// block holding the view's last record also writes the segment's padding).  A
// workgroup takes 256 consecutive sorted positions (always inside one view),
// flattens their pairs with a block scan, and for each window of 2048 output
// slots marks in LDS which record owns each slot, so consecutive threads write
// consecutive slots.
constexpr int EMIT_WIN = 2048;

__global__ __launch_bounds__(BLOCK) void k_emit(const float4 *__restrict__ ext, const uint32_t *__restrict__ order,
                                                const unsigned long long *__restrict__ counters,
                                                const uint32_t *__restrict__ poff, const uint32_t *__restrict__ ntl_s,
                                                const uint32_t *__restrict__ pbase, int64_t Kp, DevGrid g,
                                                uint32_t Dpad, uint32_t *__restrict__ pkey,
                                                uint32_t *__restrict__ pval)
{
    __shared__ unsigned char s_own[EMIT_WIN];
    __shared__ uint32_t s_pre[BLOCK];
    __shared__ int4 s_tp[BLOCK];     // ty0, a0, columns in range a, b0
    __shared__ int s_ncol[BLOCK];
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * BLOCK;
    const int64_t v = p0 / Kp, s0 = p0 - v * Kp;
    const int64_t nv = (int64_t)counters[2 * (size_t)v];
    if (s0 >= nv) return;   // uniform across the block
    const int64_t p = p0 + t;
    uint32_t nt = 0;
    int4 tp = make_int4(0, 0, 0, 0);
    int ncol = 1;
    if (s0 + t < nv) {
        nt = ntl_s[p];
        if (nt) {
            const float4 e = ext[(size_t)v * Kp + min((int64_t)order[p], Kp - 1)];
            int ty0, ty1, a0, a1, b0, b1;
            tile_rows(e.y, e.w, g.H, ty0, ty1);
            ncol = tile_cols(e.x, e.z, g.W, g.tiles_x, a0, a1, b0, b1);
            tp = make_int4(ty0, a0, a1 - a0 + 1, b0);
            if (ncol < 1) {
                ncol = 1;
                nt = 0;
            }
        }
    }
    uint32_t tot;
    const uint32_t pre = block_exclusive_scan(nt, tot, s_w);
    s_pre[t] = pre;
    s_tp[t] = tp;
    s_ncol[t] = ncol;
    const uint32_t out0 = pbase[v] + (poff[p0] - poff[(size_t)v * Kp]);
    for (uint32_t c0 = 0; c0 < tot; c0 += EMIT_WIN) {
        __syncthreads();
        const uint32_t a = max(pre, c0), b = min(pre + nt, c0 + (uint32_t)EMIT_WIN);
        for (uint32_t x = a; x < b; x++) s_own[x - c0] = (unsigned char)t;
        __syncthreads();
        const uint32_t cend = min(tot, c0 + (uint32_t)EMIT_WIN);
        for (uint32_t i = c0 + t; i < cend; i += BLOCK) {
            const int r = s_own[i - c0];
            const int4 q = s_tp[r];
            const int nc = s_ncol[r];
            const int j = (int)(i - s_pre[r]);
            const int ty = q.x + j / nc, c = j % nc;
            const int tx = c < q.z ? q.y + c : q.w + (c - q.z);
            const uint32_t o = out0 + i;
            if (o < Dpad) {
                pkey[o] = (uint32_t)(ty * g.tiles_x + tx);
                pval[o] = (uint32_t)(p0 + r);
            }
        }
    }
    if (s0 + BLOCK >= nv) {
        // this block holds the view's last record: pad the segment to a whole unit
        const uint32_t dend = out0 + tot;
        const uint32_t pend = (uint32_t)(((uint64_t)dend + SORT_TILE - 1) / SORT_TILE * SORT_TILE);
        for (uint32_t o = dend + t; o < pend && o < Dpad; o += BLOCK) pkey[o] = 0xFFFFFFFFu;
    }
}

// [start, end) of each (view, tile) list, read from the pair sort's scanned
// histogram (one 8-bit pass with the tile id as the digit): the start of digit
// d in the first block of the view's segment, and the start of digit d + 1.
// one workgroup per view: the pair sort's digit totals of the view are its
// per-tile list lengths; their exclusive scan from the view's segment start
// gives the lists' positions.  A view without pairs has empty lists (its
// totals are not read: the sort, and the clearing of its scratch, is skipped
// when a render has no pairs at all).
__global__ __launch_bounds__(BLOCK) void k_ranges_hist(const uint32_t *__restrict__ hist,
                                                       const uint32_t *__restrict__ pbase,
                                                       const uint32_t *__restrict__ pcount, int tiles,
                                                       uint2 *__restrict__ ranges)
{
    __shared__ uint32_t s_w[4];
    const int v = blockIdx.x, t = threadIdx.x;
    const uint32_t c = pcount[v] ? hist[(size_t)v * 256 + t] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(c, tot, s_w);
    if (t < tiles) {
        const uint32_t s0 = pbase[v] + ex;
        ranges[(size_t)v * tiles + t] = c ? make_uint2(s0, s0 + c) : make_uint2(0u, 0u);
    }
}

// [start, end) of each (view, tile) list in the padded pair array
__global__ __launch_bounds__(BLOCK) void k_ranges(const uint32_t *__restrict__ skey, uint32_t Dpad,
                                                  const int4 *__restrict__ segtab, int tiles,
                                                  uint2 *__restrict__ ranges)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= Dpad) return;
    const uint32_t key = skey[i];
    if (key >= (uint32_t)tiles) return;   // padding
    const int4 e = segtab[i / SORT_TILE];
    const uint32_t first = (uint32_t)e.x * SORT_TILE, end = first + (uint32_t)e.y * SORT_TILE;
    const size_t seg = (size_t)e.z * tiles + key;
    if (i == first || skey[i - 1] != key) ranges[seg].x = i;
    if (i + 1 == end || skey[i + 1] != key) ranges[seg].y = i + 1;
}

// ----------------------------------------------------------------------------
// Stage 2: radiance per (receiver, sorted position)
__global__ __launch_bounds__(BLOCK) void k_rad_direct(const float2 *__restrict__ radiance,
                                                      const uint32_t *__restrict__ order,
                                                      const unsigned long long *__restrict__ counters,
                                                      const int *__restrict__ rxview, int N, int64_t Kp,
                                                      int64_t K, float2 *__restrict__ rad)
{
    const int64_t idx = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= (int64_t)N * Kp) return;
    const int64_t j = idx / Kp, s = idx - j * Kp;
    const int v = rxview[j];
    if (s < (int64_t)counters[2 * (size_t)v]) rad[idx] = radiance[min((int64_t)order[(size_t)v * Kp + s], K - 1)];
}

// receiver ("global") term of layer 1: W1[:, :36] gamma(r_j), stored in hid_pos order
// largest |x| over the wave, folded into *dst as FP32 bits (non-negative
// floats order like their bit patterns)
__device__ __forceinline__ unsigned wave_absmax_bits(float x)
{
    unsigned b = __float_as_uint(fabsf(x));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) b = max(b, (unsigned)__shfl_xor((int)b, o));
    return b;
}

// workgroup max |x| into one of 64 slots (blockIdx % 64), so that no single
// address takes an atomic from every workgroup
__device__ __forceinline__ void block_absmax_to(float x, unsigned *slots)
{
    __shared__ unsigned s_m[BLOCK / 64];
    const unsigned b = wave_absmax_bits(x);
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = s_m[0];
        for (int w = 1; w < BLOCK / 64; w++) m = max(m, s_m[w]);
        atomicMax(slots + (blockIdx.x & 63), m);
    }
}

// MLP work item i from the per-view item offsets: view by binary search, then
// (position block, receiver block) in position-major order within the view;
// item = (view, s0, first receiver, receivers | valid positions << 8)
__device__ __forceinline__ int4 make_item(int i, const uint32_t *__restrict__ item_off,
                                          const int4 *__restrict__ vinfo, int V)
{
    int lo = 0, hi = V - 1;   // last view with item_off[v] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (item_off[mid] <= (uint32_t)i) lo = mid;
        else hi = mid - 1;
    }
    const int4 vi = vinfo[lo];   // (first receiver, receivers, visible, 0)
    const int q = i - (int)item_off[lo];
    const int nrg = (vi.y + MLP_RG - 1) / MLP_RG;
    const int sb = q / nrg, a = q - sb * nrg;
    const int s0 = sb * MLP_PAIRS;
    const int nvalid = min(MLP_PAIRS, vi.z - s0);
    const int nj = min(MLP_RG, vi.y - a * MLP_RG);
    return make_int4(lo, s0, vi.x + a * MLP_RG, nj | (nvalid << 8));
}

// Receiver ("global") term of layer 1, W1[:, :36] gamma(r_j), in hid_pos
// order; the workgroups past the receivers' expand the MLP work items.
__global__ __launch_bounds__(BLOCK) void k_mlp_global(const float *__restrict__ W1, const float *__restrict__ rx,
                                                      int N, float *__restrict__ Gp, unsigned *__restrict__ amax,
                                                      int nbg, const uint32_t *__restrict__ item_off,
                                                      const int4 *__restrict__ vinfo, int V, int nitems,
                                                      int4 *__restrict__ items)
{
    if ((int)blockIdx.x >= nbg) {
        const int i = ((int)blockIdx.x - nbg) * BLOCK + threadIdx.x;
        if (i < nitems) items[i] = make_item(i, item_off, vinfo, V);
        return;
    }
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    float acc = 0.f;
    if (idx < N * HID) {
        const int j = idx / HID, d = idx % HID;
        for (int a = 0; a < 3; a++) {
            const float r = rx[3 * j + a];
            for (int f = 0; f < 6; f++) {
                float sn, cs;
                sincosf(ldexpf(r, f), &sn, &cs);
                acc = fmaf(W1[d * MLP_IN + 12 * a + 2 * f], sn, acc);
                acc = fmaf(W1[d * MLP_IN + 12 * a + 2 * f + 1], cs, acc);
            }
        }
        Gp[(size_t)j * HID + hid_pos(d)] = acc;
    }
    block_absmax_to(acc, amax);
}

// Gaussian ("local") term of layer 1: W1[:, 36:] f_k + b1, stored in hid_pos order
// 64 Gaussians per workgroup, W1[:, 36:] and the features staged in LDS
__global__ __launch_bounds__(BLOCK) void k_mlp_local(const float *__restrict__ W1, const float *__restrict__ b1,
                                                     const float *__restrict__ feat, int64_t K,
                                                     float *__restrict__ Lp, unsigned *__restrict__ amax)
{
    __shared__ float s_w[FEAT][HID + 1];
    __shared__ float s_f[64][FEAT + 1];
    const int64_t k0 = (int64_t)blockIdx.x * 64;
    for (int i = threadIdx.x; i < HID * FEAT; i += BLOCK) {
        const int d = i / FEAT, c = i % FEAT;
        s_w[c][d] = W1[d * MLP_IN + ENC + c];
    }
    for (int i = threadIdx.x; i < 64 * FEAT; i += BLOCK) {
        const int kk = i / FEAT, c = i % FEAT;
        s_f[kk][c] = (k0 + kk < K) ? feat[(size_t)(k0 + kk) * FEAT + c] : 0.f;
    }
    __syncthreads();
    const int d = threadIdx.x & 63;
    const float bias = b1[d];
    float m = 0.f;
    for (int kk = threadIdx.x >> 6; kk < 64; kk += BLOCK / 64) {
        if (k0 + kk >= K) break;
        float acc = bias;
#pragma unroll
        for (int c = 0; c < FEAT; c++) acc = fmaf(s_w[c][d], s_f[kk][c], acc);
        Lp[(size_t)(k0 + kk) * HID + hid_pos(d)] = acc;
        m = fmaxf(m, fabsf(acc));
    }
    block_absmax_to(m, amax);
}

// Per-(receiver, Gaussian) layers 2 and 3 on FP32 MFMA (v_mfma_f32_32x32x2f32).
// One wave per work item = (view, 32 consecutive sorted positions, up to 16
// receivers of that view).  The wave computes H2^T = W2 X1^T for its 32
// pairs: A = W2 rows from LDS, B = X1 = relu(local + global), one pair per
// lane pair (lane l and l + 32 hold the two halves of the hidden units, in
// hid_of order), so the accumulator leaves each lane with 32 of the 64 hidden
// outputs of its own pair.  Layer 3 (64 -> 2) is then a per-lane dot product
// plus one exchange between the two lane halves.
__global__ __launch_bounds__(BLOCK) void k_mlp_pairs_f32(const float *__restrict__ Lp, const float *__restrict__ Gp,
                                                     const float *__restrict__ w2a,
                                                     const float4 *__restrict__ tab, const float *__restrict__ b3,
                                                     const uint32_t *__restrict__ order,
                                                     const int4 *__restrict__ items, int nitems, int64_t Kp,
                                                     int64_t K, const unsigned long long *__restrict__ counters,
                                                     float2 *__restrict__ rad)
{
    __shared__ float s_w2a[2 * 32 * 64];
    __shared__ float4 s_tab[2 * 2 * 16];
    for (int i = threadIdx.x; i < 2 * 32 * 64; i += BLOCK) s_w2a[i] = w2a[i];
    if (threadIdx.x < 64) s_tab[threadIdx.x] = tab[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, h = lane >> 5, pl = lane & 31;
    const float b30 = b3[0], b31 = b3[1];
    // persistent waves: the workgroup stages W2 once and walks many work items
    for (int item = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); item < nitems; item += gridDim.x * (BLOCK / 64)) {
    const int4 it = items[item];
    const int view = it.x, s0 = it.y, j0 = it.z, nj = it.w & 255;
    const int64_t nv = (int64_t)counters[2 * (size_t)view];
    const int64_t s = s0 + pl;
    const bool valid = s < nv;
    const uint32_t k = (uint32_t)min((int64_t)order[(size_t)view * Kp + (valid ? s : s0)], K - 1);
    float l[32];
    {
        const float4 *src = reinterpret_cast<const float4 *>(Lp + (size_t)k * HID + h * 32);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const float4 x = src[q];
            l[4 * q] = x.x; l[4 * q + 1] = x.y; l[4 * q + 2] = x.z; l[4 * q + 3] = x.w;
        }
    }
    for (int jj = 0; jj < nj; jj++) {
        const int j = j0 + jj;
        // an index the compiler cannot prove loop-invariant: keeps the layer-3
        // and bias constants in LDS instead of ~100 hoisted registers
        int z0 = 0;
        asm volatile("" : "+v"(z0));
        const float4 *tabh = s_tab + h * 32 + z0;
        float x1[32];
        const float4 *gs = reinterpret_cast<const float4 *>(Gp + (size_t)j * HID + h * 32);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const float4 gv = gs[q];
            x1[4 * q] = fmaxf(l[4 * q] + gv.x, 0.f);
            x1[4 * q + 1] = fmaxf(l[4 * q + 1] + gv.y, 0.f);
            x1[4 * q + 2] = fmaxf(l[4 * q + 2] + gv.z, 0.f);
            x1[4 * q + 3] = fmaxf(l[4 * q + 3] + gv.w, 0.f);
        }
        floatx16 acc0, acc1;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            acc0[r] = tabh[r].z;
            acc1[r] = tabh[16 + r].z;
        }
#pragma unroll
        for (int t = 0; t < 32; t++) {
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(s_w2a[(0 * 32 + t) * 64 + lane], x1[t], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(s_w2a[(1 * 32 + t) * 64 + lane], x1[t], acc1, 0, 0, 0);
        }
        float o0 = 0.f, o1 = 0.f;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float4 ta = tabh[r];
            const float4 tb = tabh[16 + r];
            const float ha = fmaxf(acc0[r], 0.f), hb = fmaxf(acc1[r], 0.f);
            o0 = fmaf(ta.x, ha, o0);
            o1 = fmaf(ta.y, ha, o1);
            o0 = fmaf(tb.x, hb, o0);
            o1 = fmaf(tb.y, hb, o1);
        }
        o0 += __shfl_xor(o0, 32);
        o1 += __shfl_xor(o1, 32);
        if (h == 0 && valid) rad[(size_t)j * Kp + s] = make_float2(o0 + b30, o1 + b31);
    }
    }
}

// The same layers with layer 2 on FP16 MFMA (v_mfma_f32_32x32x16_f16) in split
// precision: every FP32 operand x is carried as an FP16 pair hi = fp16(x),
// lo = fp16(x - hi), and W2 x1 is summed as Wlo xhi + Whi xlo + Whi xhi in an
// FP32 accumulator, which leaves a relative error near 2^-21 per product (the
// dropped Wlo xlo term and the rounding of the lo halves) at about a sixth of
// the matrix-core time of the FP32 instruction.  W2 arrives pre-split and
// pre-scaled by 2^wexp and stays in registers for the life of the wave.  The
// layer-1 activations are split unscaled while the largest possible one,
// max|local| + max|global|, is below 2^15; beyond that a uniform branch scales
// them by a power of two first, so no operand leaves the FP16 range.
// one 64-float row stored in hid_pos order: lane half h takes its 32 values
__device__ __forceinline__ void load_half_row(const float *__restrict__ base, size_t row, int h, float (&v)[32])
{
    const float4 *src = reinterpret_cast<const float4 *>(base + row * HID + h * 32);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const float4 x = src[q];
        v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
    }
}

// Work item descriptor: (view, first sorted position s0, first receiver j0,
// receivers | valid positions << 8).
__device__ __forceinline__ int4 read_desc(const int4 &batch, int lane_idx)
{
    return make_int4(__builtin_amdgcn_readlane(batch.x, lane_idx), __builtin_amdgcn_readlane(batch.y, lane_idx),
                     __builtin_amdgcn_readlane(batch.z, lane_idx), __builtin_amdgcn_readlane(batch.w, lane_idx));
}

// Each wave walks its items n = 0, 1, ... (global index i0 + n S, S = waves in
// the grid) as a software pipeline: descriptors arrive 64 at a time, one per
// lane, and are read out as wave-uniform values; the sorted-order entries of
// item n + 2 are loaded while item n is computed; the local rows of item n + 1
// and every next receiver's global row are loaded right after the current
// unit's activations are split, so the loads overlap the unit's MFMA work.
template <bool SCALED>
__device__ __forceinline__ void mlp_pairs_walk(const float *__restrict__ Lp, const float *__restrict__ Gp,
                                               const half8 *s_w2h, const float4 *s_b2, const float4 *s_w3,
                                               float b30, float b31, float sx,
                                               const uint32_t *__restrict__ order, const int4 *__restrict__ items,
                                               int nitems, int64_t Kp, int64_t K, float2 *__restrict__ rad)
{
    const int lane = threadIdx.x & 63, h = lane >> 5, pl = lane & 31;
    const float isx = 1.f / sx;
    const int S = gridDim.x * (BLOCK / 64);
    const int i0 = blockIdx.x * (BLOCK / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i0 >= nitems) return;
    const int nmine = (nitems - i0 + S - 1) / S;
    // descriptors of items base .. base + 63 of this wave, one per lane
    int base = 0;
    const int4 zero4 = make_int4(0, 0, 0, 0);
    int4 batch = lane < nmine ? items[i0 + lane * S] : zero4;
    int4 dc = read_desc(batch, 0);
    int4 dn = nmine > 1 ? read_desc(batch, 1) : dc;
    // sorted positions s0 + pl exist for every item (s0 is a multiple of 32
    // below the view's visible count and the sorted order has Kp >= that
    // rounded up to 4096 entries); entries are clamped, stores check validity
    uint32_t kA = order[(size_t)dn.x * Kp + dn.y + pl];
    float l[32], g[32];
    load_half_row(Lp, min((int64_t)order[(size_t)dc.x * Kp + dc.y + pl], K - 1), h, l);
    load_half_row(Gp, (size_t)dc.z, h, g);
    for (int n = 0; n < nmine; n++) {
        int4 dnn = dn;
        uint32_t kB = kA;
        if (n + 2 < nmine) {
            if (n + 2 - base >= 64) {
                base = n + 2;
                batch = base + lane < nmine ? items[i0 + (base + lane) * S] : zero4;
            }
            dnn = read_desc(batch, n + 2 - base);
            kB = order[(size_t)dnn.x * Kp + dnn.y + pl];
        }
        const int nj = dc.w & 255;
        const bool valid = pl < (dc.w >> 8);
        const int64_t s = dc.y + pl;
        const bool more = n + 1 < nmine;
        for (int jj = 0; jj < nj; jj++) {
            int z0 = 0;
            asm volatile("" : "+v"(z0));
            const float4 *b2h = s_b2 + h * 8 + z0;
            const float4 *w3h = s_w3 + h * 16 + z0;
            half8 bh[4], bl[4];
#pragma unroll
            for (int t = 0; t < 32; t++) {
                float v = fmaxf(l[t] + g[t], 0.f);
                if (SCALED) v *= sx;
                const _Float16 hi = (_Float16)v;
                bh[t >> 3][t & 7] = hi;
                bl[t >> 3][t & 7] = (_Float16)(v - (float)hi);
            }
            const bool last = jj + 1 == nj;
            if (last && more) load_half_row(Lp, min((int64_t)kA, K - 1), h, l);
            load_half_row(Gp, (size_t)(last ? (more ? dn.z : dc.z) : dc.z + jj + 1), h, g);
            floatx16 acc0, acc1;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const float4 u = b2h[r], w = b2h[4 + r];
                acc0[4 * r] = u.x; acc0[4 * r + 1] = u.y; acc0[4 * r + 2] = u.z; acc0[4 * r + 3] = u.w;
                acc1[4 * r] = w.x; acc1[4 * r + 1] = w.y; acc1[4 * r + 2] = w.z; acc1[4 * r + 3] = w.w;
            }
            if (SCALED) {
                acc0 *= sx;
                acc1 *= sx;
            }
            // small cross terms first, then the leading product
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const half8 h0 = s_w2h[(0 * 4 + q) * 64 + lane + z0];
                const half8 h1 = s_w2h[(1 * 4 + q) * 64 + lane + z0];
                const half8 l0 = s_w2h[(2 * 4 + q) * 64 + lane + z0];
                const half8 l1 = s_w2h[(3 * 4 + q) * 64 + lane + z0];
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(l0, bh[q], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(l1, bh[q], acc1, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(h0, bl[q], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(h1, bl[q], acc1, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const half8 h0 = s_w2h[(0 * 4 + q) * 64 + lane + z0];
                const half8 h1 = s_w2h[(1 * 4 + q) * 64 + lane + z0];
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(h0, bh[q], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(h1, bh[q], acc1, 0, 0, 0);
            }
            float o0 = 0.f, o1 = 0.f;
#pragma unroll
            for (int r = 0; r < 8; r++) {
                const float4 ta = w3h[r];       // W3 columns of acc0 registers 2r, 2r + 1
                const float4 tb = w3h[8 + r];   // and of acc1
                const float a0 = fmaxf(acc0[2 * r], 0.f), a1 = fmaxf(acc0[2 * r + 1], 0.f);
                const float c0 = fmaxf(acc1[2 * r], 0.f), c1 = fmaxf(acc1[2 * r + 1], 0.f);
                o0 = fmaf(ta.x, a0, o0);
                o1 = fmaf(ta.y, a0, o1);
                o0 = fmaf(ta.z, a1, o0);
                o1 = fmaf(ta.w, a1, o1);
                o0 = fmaf(tb.x, c0, o0);
                o1 = fmaf(tb.y, c0, o1);
                o0 = fmaf(tb.z, c1, o0);
                o1 = fmaf(tb.w, c1, o1);
            }
            o0 += __shfl_xor(o0, 32);
            o1 += __shfl_xor(o1, 32);
            if (SCALED) {
                o0 *= isx;
                o1 *= isx;
            }
            if (h == 0 && valid) rad[(size_t)(dc.z + jj) * Kp + s] = make_float2(o0 + b30, o1 + b31);
        }
        dc = dn;
        dn = dnn;
        kA = kB;
    }
}

__global__ __launch_bounds__(BLOCK) void k_mlp_pairs(const float *__restrict__ Lp, const float *__restrict__ Gp,
                                                     const half8 *__restrict__ w2h,
                                                     const float4 *__restrict__ tab, const float *__restrict__ b3,
                                                     const uint32_t *__restrict__ order,
                                                     const int4 *__restrict__ items, int nitems, int64_t Kp,
                                                     int64_t K, const unsigned long long *__restrict__ counters,
                                                     const unsigned *__restrict__ amax, float2 *__restrict__ rad)
{
    // per lane half h: layer-2 bias of accumulator registers (acc0 r, acc1 r)
    // as 8 float4, and layer-3 weights (W3[0][d], W3[1][d]) of register pairs
    // as 16 float4
    __shared__ float4 s_b2[2 * 8];
    __shared__ float4 s_w3[2 * 16];
    // split W2, [hi mb0, hi mb1, lo mb0, lo mb1][q][lane] as in w2h
    __shared__ half8 s_w2h[16 * 64];
    if (threadIdx.x < 64) {
        const int hh = threadIdx.x >> 5, i = threadIdx.x & 31;   // (h, mb, r) = (hh, i / 16, i % 16)
        const float4 e = tab[hh * 32 + i];
        reinterpret_cast<float *>(s_b2)[hh * 32 + i] = e.z;
        reinterpret_cast<float2 *>(s_w3)[hh * 32 + i] = make_float2(e.x, e.y);
    }
    for (int i = threadIdx.x; i < 16 * 64; i += BLOCK) s_w2h[i] = w2h[i];
    __syncthreads();
    const float b30 = b3[0], b31 = b3[1];
    const int lane = threadIdx.x & 63;
    // largest layer-1 term magnitudes, spread over 64 slots each
    unsigned mb = max(amax[lane], amax[64 + lane]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mb = max(mb, (unsigned)__shfl_xor((int)mb, o));
    const float bound = 2.f * __uint_as_float(mb);
    if (bound < 32768.f) {
        mlp_pairs_walk<false>(Lp, Gp, s_w2h, s_b2, s_w3, b30, b31, 1.f, order, items, nitems, Kp, K, rad);
    } else {
        int e = 0;
        frexpf(bound, &e);   // bound < 2^e
        const float sx = (e > 15 && e < 128) ? ldexpf(1.f, 15 - e) : 1.f;
        mlp_pairs_walk<true>(Lp, Gp, s_w2h, s_b2, s_w3, b30, b31, sx, order, items, nitems, Kp, K, rad);
    }
}

// ----------------------------------------------------------------------------
// Stage 3: front-to-back compositing.  One workgroup per (tile, chunk of R
// receivers of one view); one pixel per thread, each wave an 8 x 8 sub-tile.
// Batches of 256 list entries (record + R radiance values) are staged in LDS;
// while staging, each entry's conservative support box is tested against the
// four sub-tiles and a ballot/prefix pass builds, per wave, the ordered list of
// entries that can reach it, so a wave walks only those.  Every lane keeps its
// own transmittance; a wave stops once all its lanes have terminated and the
// workgroup stops staging once all its waves have.
template <int R>
__global__ __launch_bounds__(BLOCK) void k_blend_fwd(const float4 *__restrict__ srec,
                                                     const uint32_t *__restrict__ pval,
                                                     const uint2 *__restrict__ ranges,
                                                     const float2 *__restrict__ rad,
                                                     const int4 *__restrict__ chunks, int64_t Kp, DevGrid g,
                                                     float *__restrict__ C, float *__restrict__ Tfin,
                                                     int *__restrict__ nlast, float *__restrict__ part,
                                                     unsigned long long *__restrict__ stats)
{
    __shared__ BlendStage st;
    __shared__ float2 s_rad[R][BLOCK];
    __shared__ float s_red[4][R][3];

    const int tile = blockIdx.x;
    const int4 ch = chunks[blockIdx.y];
    const int view = ch.x, j0 = ch.y, nrx = ch.z, tslot = ch.w;
    const int ty = tile / g.tiles_x, tx = tile - ty * g.tiles_x;
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
    const int row = ty * TILE + 8 * (wv >> 1) + (lane >> 3), col = tx * TILE + 8 * (wv & 1) + (lane & 7);
    const bool inside = row < g.H && col < g.W;
    const float rowf = (float)row, colf = (float)col;
    const float Wf = (float)g.W, halfW = 0.5f * (float)g.W;
    const uint2 rg = ranges[(size_t)view * g.tiles + tile];
    const int64_t view_end = ((int64_t)view + 1) * Kp;

    float T = 1.f;
    float2 acc[R];
#pragma unroll
    for (int r = 0; r < R; r++) acc[r] = make_float2(0.f, 0.f);
    int last = 0;
    uint32_t ncomp = 0;   // composited entries of this pixel
    bool done = !inside;

    for (uint32_t base = rg.x; base < rg.y; base += BLOCK) {
        const uint32_t cnt = min((uint32_t)BLOCK, rg.y - base);
        __syncthreads();
        uint32_t p = 0;
        if ((uint32_t)t < cnt) {
            p = min(pval[base + t], (uint32_t)(view_end - 1));
            const int64_t s = max((int64_t)p - (int64_t)view * Kp, (int64_t)0);
#pragma unroll
            for (int r = 0; r < R; r++)
                s_rad[r][t] = (r < nrx) ? rad[(size_t)(j0 + r) * Kp + s] : make_float2(0.f, 0.f);
        }
        stage_batch(st, srec, p, (uint32_t)t < cnt, tx, ty, g);
        if (!done) {
            const int n = st.len[wv];
            for (int i = 0; i < n; i++) {
                const int e = st.list[wv][i];
                const float4 r0 = st.r0[e];
                const float4 r1 = st.r1[e];
                float du = (colf - r0.x) - r0.y;
                if (st.wide[e]) {
                    if (du >= halfW) du -= Wf;
                    else if (du < -halfW) du += Wf;
                }
                const float dv = (rowf - r0.z) - r0.w;
                const float w = fminf(W_MAX, __builtin_amdgcn_exp2f(blend_exponent(du, dv, r1)));
                if (w < ALPHA_MIN) continue;
                const float tw = T * w;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const float2 sv = s_rad[r][e];
                    acc[r].x = fmaf(tw, sv.x, acc[r].x);
                    acc[r].y = fmaf(tw, sv.y, acc[r].y);
                }
                T = T * (1.f - w);
                last = (int)(base - rg.x) + e + 1;
                ncomp++;
                if (T < T_EPS) {
                    done = true;
                    break;
                }
            }
        }
        if (__syncthreads_and(done ? 1 : 0)) break;
    }

    const size_t P = (size_t)g.H * g.W;
    const size_t pix = (size_t)row * g.W + col;
    if (inside) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (r < nrx) {
                C[((size_t)(j0 + r) * 2) * P + pix] = acc[r].x;
                C[((size_t)(j0 + r) * 2 + 1) * P + pix] = acc[r].y;
            }
        }
        if (tslot >= 0) {
            Tfin[(size_t)tslot * P + pix] = T;
            nlast[(size_t)tslot * P + pix] = last;
        }
    }
    // per-tile partial sums: power, Re, Im (fixed-order reduction)
#pragma unroll
    for (int r = 0; r < R; r++) {
        const float pw = wave_sum_f32(acc[r].x * acc[r].x + acc[r].y * acc[r].y);
        const float sr = wave_sum_f32(acc[r].x);
        const float si = wave_sum_f32(acc[r].y);
        if (lane == 0) {
            s_red[wv][r][0] = pw;
            s_red[wv][r][1] = sr;
            s_red[wv][r][2] = si;
        }
    }
    const uint32_t nc = wave_sum_u32(ncomp);
    if (lane == 0) st.wcnt[0][wv] = nc;
    __syncthreads();
    if (t < R * 3) {
        const int r = t / 3, c = t % 3;
        if (r < nrx) {
            const float v = ((s_red[0][r][c] + s_red[1][r][c]) + s_red[2][r][c]) + s_red[3][r][c];
            part[((size_t)(j0 + r) * g.tiles + tile) * 3 + c] = v;
        }
    }
    // composited (pixel, entry) pairs: per chunk pixel and per receiver pixel,
    // spread over STAT_SLOTS counters
    if (t == 0) {
        const unsigned long long n = (unsigned long long)st.wcnt[0][0] + st.wcnt[0][1] + st.wcnt[0][2] +
                                     st.wcnt[0][3];
        if (n) {
            const unsigned slot = (blockIdx.x + blockIdx.y * gridDim.x) % STAT_SLOTS;
            atomicAdd(stats + slot, n);
            atomicAdd(stats + STAT_SLOTS + slot, n * (unsigned long long)nrx);
        }
    }
}

// one wave per receiver; lanes take tiles in a fixed stride, then a fixed
// butterfly, so the result does not depend on scheduling
__global__ __launch_bounds__(BLOCK) void k_reduce_out(const float *__restrict__ part, int N, int tiles,
                                                      float *__restrict__ power, float *__restrict__ csum)
{
    const int j = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= N) return;
    double pw = 0, sr = 0, si = 0;
    for (int t = lane; t < tiles; t += 64) {
        const float *p = part + ((size_t)j * tiles + t) * 3;
        pw += p[0];
        sr += p[1];
        si += p[2];
    }
    for (int off = 32; off > 0; off >>= 1) {
        pw += __shfl_xor(pw, off);
        sr += __shfl_xor(sr, off);
        si += __shfl_xor(si, off);
    }
    if (lane == 0) {
        if (power) power[j] = (float)pw;
        if (csum) {
            csum[2 * j] = (float)sr;
            csum[2 * j + 1] = (float)si;
        }
    }
}

// ============================================================================
// host-side launch wrappers
static inline unsigned nblk(size_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

bool grow(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.cap >= bytes) return true;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return false;
        }
        want = bytes;
    }
    b.cap = want;
    return true;
}

void release(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned blocks = (unsigned)std::min<size_t>(nblk(n), 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(BLOCK), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_project(const Scene &sc, const float *centres, int V, int64_t Kp, const DevGrid &g,
                          Workspace &ws, hipStream_t st)
{
    const int vchunk = V <= 4 ? 1 : 4;
    dim3 grid((unsigned)(Kp / BLOCK), (unsigned)((V + vchunk - 1) / vchunk));
    hipLaunchKernelGGL(k_project, grid, dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K, Kp, centres, V, vchunk, g,
                       ws.rec.as<float4>(), ws.ext.as<float4>(), ws.rawkey.as<uint32_t>(), ws.opac.as<float>(),
                       ws.ntl.as<uint32_t>(), ws.skey[0].as<uint32_t>(), ws.sval[0].as<uint32_t>(),
                       ws.counters.as<unsigned long long>());
    return hipGetLastError();
}

// Scratch buffers are sized by the caller before any work that may still be in
// flight uses them (grow() frees the old buffer).  Small arrays are scanned by
// one workgroup in a single launch.
hipError_t scan_exclusive_u32(DevBuf &scan_tmp, const uint32_t *in, uint32_t *out, uint32_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    if (n <= SMALL_SCAN) {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, st, in, out, n);
        return hipGetLastError();
    }
    const uint32_t nb = (n + SORT_TILE - 1) / SORT_TILE;
    if (scan_tmp.cap < (size_t)nb * 4) return hipErrorOutOfMemory;
    uint32_t *bs = scan_tmp.as<uint32_t>();
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(BLOCK), 0, st, in, n, bs);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, st, bs, bs, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(BLOCK), 0, st, in, n, bs, out);
    return hipGetLastError();
}

hipError_t launch_gather(Workspace &ws, int V, int64_t Kp, hipStream_t st)
{
    const int64_t total = (int64_t)V * Kp;
    hipLaunchKernelGGL(k_gather, dim3(nblk(total)), dim3(BLOCK), 0, st, ws.rec.as<float4>(), ws.ntl.as<uint32_t>(),
                       ws.sval[ws.sorted_buf].as<uint32_t>(), ws.counters.as<unsigned long long>(), Kp, total,
                       ws.srec.as<float4>(), ws.ntl_s.as<uint32_t>());
    return hipGetLastError();
}

hipError_t launch_emit(Workspace &ws, int V, int64_t Kp, const DevGrid &g, hipStream_t st)
{
    const int64_t total = (int64_t)V * Kp;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)(total / BLOCK)), dim3(BLOCK), 0, st, ws.ext.as<float4>(),
                       ws.sval[ws.sorted_buf].as<uint32_t>(), ws.counters.as<unsigned long long>(),
                       ws.poff.as<uint32_t>(), ws.ntl_s.as<uint32_t>(), ws.d_pbase, Kp, g,
                       (uint32_t)ws.Dpad, ws.pkey[0].as<uint32_t>(), ws.pval[0].as<uint32_t>());
    return hipGetLastError();
}

hipError_t launch_ranges(Workspace &ws, const DevGrid &g, hipStream_t st)
{
    const size_t nr = (size_t)ws.V * g.tiles;
    if (g.tiles <= 255) {
        // one 8-bit pass: ranges straight from the scanned histogram
        hipLaunchKernelGGL(k_ranges_hist, dim3((unsigned)ws.V), dim3(BLOCK), 0, st, ws.hist_b.as<uint32_t>(),
                           ws.d_pbase, ws.d_pcount, g.tiles, ws.ranges.as<uint2>());
        return hipGetLastError();
    }
    hipError_t e = launch_fill_u32(ws.ranges.as<uint32_t>(), 0u, nr * 2, st);
    if (e != hipSuccess || ws.Dpad == 0) return e;
    hipLaunchKernelGGL(k_ranges, dim3(nblk((size_t)ws.Dpad)), dim3(BLOCK), 0, st,
                       ws.pkey[ws.pairs_buf].as<uint32_t>(), (uint32_t)ws.Dpad, ws.d_segtab, g.tiles,
                       ws.ranges.as<uint2>());
    return hipGetLastError();
}

hipError_t launch_rad_direct(const Scene &sc, Workspace &ws, hipStream_t st)
{
    const int64_t n = (int64_t)ws.N * ws.Kp;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rad_direct, dim3(nblk(n)), dim3(BLOCK), 0, st, sc.rad.as<float2>(),
                       ws.sval[ws.sorted_buf].as<uint32_t>(), ws.counters.as<unsigned long long>(),
                       ws.d_rxview, ws.N, ws.Kp, ws.K, ws.rad.as<float2>());
    return hipGetLastError();
}

// render statistics after the activation-bound slots: STAT_SLOTS u64 of
// composited pairs per chunk pixel, then STAT_SLOTS per receiver pixel
unsigned long long *stat_words(Workspace &ws)
{
    return ws.counters.as<unsigned long long>() + (size_t)2 * ws.V + AMAX_SLOTS / 2;
}

// the activation-bound slots after the per-view counters: 64 for the
// receivers' layer-1 terms, then 64 for the Gaussians'
static unsigned *amax_words(Workspace &ws)
{
    return ws.counters.as<uint32_t>() + (size_t)4 * ws.V;
}

hipError_t launch_mlp_global(const Mlp &m, Workspace &ws, hipStream_t st)
{
    const unsigned nbg = (unsigned)nblk((size_t)ws.N * HID);
    const unsigned nbi = (unsigned)nblk((size_t)ws.n_items);
    if (nbg + nbi > 0)
        hipLaunchKernelGGL(k_mlp_global, dim3(nbg + nbi), dim3(BLOCK), 0, st, m.raw.as<float>(), ws.rxpos_p, ws.N,
                           ws.Gp.as<float>(), amax_words(ws), (int)nbg, ws.d_item_off, ws.d_vinfo, ws.V, ws.n_items,
                           ws.items.as<int4>());
    return hipGetLastError();
}

hipError_t launch_mlp_local(const Scene &sc, const Mlp &m, Workspace &ws, hipStream_t st)
{
    const float *raw = m.raw.as<float>();
    if (sc.K > 0)
        hipLaunchKernelGGL(k_mlp_local, dim3((unsigned)((sc.K + 63) / 64)), dim3(BLOCK), 0, st, raw,
                           raw + HID * MLP_IN, sc.feat.as<float>(), sc.K, ws.Lp.as<float>(), amax_words(ws) + 64);
    return hipGetLastError();
}

hipError_t launch_mlp_pairs(const Mlp &m, Workspace &ws, hipStream_t st)
{
    const float *raw = m.raw.as<float>();
    const float *b3 = raw + HID * MLP_IN + HID + HID * HID + HID + 2 * HID;
    if (ws.n_items > 0) {
        const unsigned blocks = (unsigned)std::min((ws.n_items + 3) / 4, 256 * 8);
        if (m.fp32)
            hipLaunchKernelGGL(k_mlp_pairs_f32, dim3(blocks), dim3(BLOCK), 0, st, ws.Lp.as<float>(),
                               ws.Gp.as<float>(), m.w2a.as<float>(), m.tab.as<float4>(), b3,
                               ws.sval[ws.sorted_buf].as<uint32_t>(), ws.items.as<int4>(), ws.n_items, ws.Kp, ws.K,
                               ws.counters.as<unsigned long long>(), ws.rad.as<float2>());
        else
            hipLaunchKernelGGL(k_mlp_pairs, dim3(blocks), dim3(BLOCK), 0, st, ws.Lp.as<float>(), ws.Gp.as<float>(),
                               m.w2h.as<half8>(), m.tabh.as<float4>(), b3, ws.sval[ws.sorted_buf].as<uint32_t>(),
                               ws.items.as<int4>(), ws.n_items, ws.Kp, ws.K, ws.counters.as<unsigned long long>(),
                               amax_words(ws), ws.rad.as<float2>());
    }
    return hipGetLastError();
}

template <int R>
static void blend_launch(Workspace &ws, float *C, hipStream_t st)
{
    dim3 grid((unsigned)ws.g.tiles, (unsigned)ws.n_chunks);
    hipLaunchKernelGGL(k_blend_fwd<R>, grid, dim3(BLOCK), 0, st, ws.srec.as<float4>(),
                       ws.pval[ws.pairs_buf].as<uint32_t>(), ws.ranges.as<uint2>(), ws.rad.as<float2>(),
                       ws.d_chunks, ws.Kp, ws.g, C, ws.Tfin.as<float>(), ws.nlast.as<int>(),
                       ws.part.as<float>(), stat_words(ws));
}

hipError_t launch_blend_fwd(Workspace &ws, float *C, hipStream_t st)
{
    if (ws.n_chunks == 0) return hipSuccess;
    switch (ws.R) {
    case 1: blend_launch<1>(ws, C, st); break;
    case 2: blend_launch<2>(ws, C, st); break;
    case 4: blend_launch<4>(ws, C, st); break;
    case 8: blend_launch<8>(ws, C, st); break;
    default: blend_launch<16>(ws, C, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_outputs(Workspace &ws, float *power, float *csum, hipStream_t st)
{
    if (ws.N == 0 || (!power && !csum)) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_out, dim3((unsigned)((ws.N + 3) / 4)), dim3(BLOCK), 0, st, ws.part.as<float>(), ws.N,
                       ws.g.tiles, power, csum);
    return hipGetLastError();
}

}  // namespace rxgs
