// Device helpers shared by the forward and backward kernels of librxgs.
#pragma once

#include "rxgs_internal.h"

namespace rxgs {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int count_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of a wave whose 8-bit keys equal this lane's, among the lanes in
// `m`: eight ballots, one per key bit; a lane keeps the lanes whose bit
// agrees with its own (m & (bb xnor own bit), one three-input bit operation
// per 32-lane half; truth table 0x90 over (m, bb, own bit)).
__device__ __forceinline__ uint64_t match_key8(uint32_t d, uint64_t m)
{
    uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
#pragma unroll
    for (int bt = 0; bt < 8; bt++) {
        const uint32_t own = (uint32_t)(((int32_t)(d << (31 - bt))) >> 31);   // all ones if bit bt is set
        const uint64_t bb = __ballot(own != 0u);
        lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)bb, own, 0x90);
        hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(bb >> 32), own, 0x90);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Blend exponent of one (pixel, record): log2 of o exp(-q/2), with the record
// holding (-a/2, -b, -c/2) log2(e) and log2(o).  Written with explicit fmaf so
// that the forward and the backward evaluate bit-identical weights.
__device__ __forceinline__ float blend_exponent(float du, float dv, const float4 &r1)
{
    return fmaf(du, fmaf(r1.x, du, r1.y * dv), fmaf(r1.z * dv, dv, r1.w));
}

// Hidden-unit order of the MLP on MFMA.  Lane half h (lanes 0-31 / 32-63) at
// step t (0..31) handles hidden unit hid_of(h, t); the same map gives the rows
// an MFMA 32x32 accumulator leaves in lane half h, register r of block b
// (t = 16 b + r), so layer-2 inputs, layer-2 outputs and the backward's
// layer-1 gradients line up register by register.
__host__ __device__ __forceinline__ int hid_of(int h, int t)
{
    return 8 * ((t & 15) >> 2) + 4 * h + (t & 3) + 32 * (t >> 4);
}
// position of hidden unit d in a row stored in that order (h * 32 + t)
__host__ __device__ __forceinline__ int hid_pos(int d)
{
    const int h = (d & 7) >> 2;
    const int t = 16 * (d >> 5) + 4 * ((d & 31) >> 3) + (d & 3);
    return h * 32 + t;
}

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
    // c0 mod W; c0 lies in (-W, W) for every box on the grid, other values
    // take the general form
    int m = c0 < 0 ? c0 + W : c0;
    if ((unsigned)m >= (unsigned)W) m = ((c0 % W) + W) % W;
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

// index of tile (ty, tx) in the enumeration the pair emission uses for a
// record covering rows ty0.. and the column ranges a0..a1, b0..b1: row-major,
// the first column range before the second
__device__ __forceinline__ int tile_rank(int ty, int tx, int ty0, int a0, int a1, int b0, int b1)
{
    const int na = a1 - a0 + 1, nc = na + (b1 - b0 + 1);
    const int cx = (tx >= a0 && tx <= a1) ? tx - a0 : na + (tx - b0);
    return (ty - ty0) * nc + cx;
}

// DPP move (row_shr, row_bcast, ...) with masked-off or out-of-row lanes reading 0
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_shift(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK,
                                                                 0xf, false));
}

// Sum over each 16-lane row; lanes 15, 31, 47 and 63 hold the four sums.
__device__ __forceinline__ float row_sum(float x)
{
    x += dpp_shift<0x111, 0xf>(x);   // row_shr:1
    x += dpp_shift<0x112, 0xf>(x);   // row_shr:2
    x += dpp_shift<0x114, 0xf>(x);   // row_shr:4
    x += dpp_shift<0x118, 0xf>(x);   // row_shr:8
    return x;
}

// Sum over each 32-lane half of the wave; lanes 31 and 63 hold the two sums.
__device__ __forceinline__ float half_wave_sum(float x)
{
    x += dpp_shift<0x111, 0xf>(x);   // row_shr:1
    x += dpp_shift<0x112, 0xf>(x);   // row_shr:2
    x += dpp_shift<0x114, 0xf>(x);   // row_shr:4
    x += dpp_shift<0x118, 0xf>(x);   // row_shr:8
    x += dpp_shift<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    return x;
}

// Sum over the whole wave; lane 63 holds the sum.
__device__ __forceinline__ float wave_sum_last(float x)
{
    x = half_wave_sum(x);
    x += dpp_shift<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// ---------------------------------------------------------------------------
// LDS staging of one batch of a tile's list for the blend kernels.
struct BlendStage {
    float4 r0[BLOCK];            // (floor u shifted near the tile, frac u, floor v, frac v)
    float4 r1[BLOCK];            // exponent coefficients and log2 opacity
    uint32_t p[BLOCK];           // sorted position of the entry
    int wide[BLOCK];             // azimuth offsets inside the tile may need wrapping
    unsigned short list[4][BLOCK];  // per wave: entries (in list order) that can reach its sub-tile
    int len[4];
    int wrap[4];                 // per wave: its list holds an entry that needs azimuth wrapping
    int wcnt[4][4];
    int ncnt[4][4];              // per source wave and sub-tile: entries below a position prefix
};

// Conservative sub-tile mask of one record: bit w set when the box around the
// ellipse {ex >= log2(1/255)} meets wave w's 8 x 8 sub-tile.
__device__ __forceinline__ int subtile_mask(const float4 &r0, const float4 &r1, int wide, int tx, int ty)
{
    if (wide) return 0xF;
    float lo = r1.w - (-7.99435343685886f);   // log2 o - log2(1/255)
    if (!(lo >= -1e-3f)) return 0;
    lo = fmaxf(lo, 0.f) + 1e-3f;
    const float muu = -r1.x, muv = -0.5f * r1.y, mvv = -r1.z;
    const float det = muu * mvv - muv * muv;
    if (!(det > 0.f)) return 0xF;
    const float ru = sqrtf(lo * mvv / det) * 1.001f + 0.05f;
    const float rv = sqrtf(lo * muu / det) * 1.001f + 0.05f;
    const float u = r0.x + r0.y, v = r0.z + r0.w;
    const float c0 = (float)(tx * TILE), r0f = (float)(ty * TILE);
    int m = 0;
#pragma unroll
    for (int w = 0; w < 4; w++) {
        const float cl = c0 + 8.f * (float)(w & 1), rl = r0f + 8.f * (float)(w >> 1);
        const bool hit = (u + ru >= cl) && (u - ru <= cl + 7.f) && (v + rv >= rl) && (v - rv <= rl + 7.f);
        m |= hit ? (1 << w) : 0;
    }
    return m;
}

// Stage the batch entry of this thread (if `has`) and build the per-wave lists.
// All threads of the block must call it.
__device__ __forceinline__ void stage_batch(BlendStage &st, const float4 *__restrict__ srec, uint32_t p, bool has,
                                            int tx, int ty, const DevGrid &g, bool nearp = true)
{
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    int m = 0;
    if (has) {
        float4 r0 = srec[2 * (size_t)p];
        const float4 r1 = srec[2 * (size_t)p + 1];
        const float Wf = (float)g.W, halfW = 0.5f * (float)g.W;
        const float tcol = (float)(tx * TILE) + 7.5f;
        // representative of the azimuth closest to this tile's centre
        const float sh = rintf((tcol - r0.x) / Wf);
        r0.x = fmaf(sh, Wf, r0.x);
        const int wide = fabsf(tcol - (r0.x + r0.y)) >= halfW - 9.0f;
        st.r0[t] = r0;
        st.r1[t] = r1;
        st.p[t] = p;
        st.wide[t] = wide;
        m = subtile_mask(r0, r1, wide, tx, ty);
    }
    uint64_t bal[4], nbal[4];
#pragma unroll
    for (int b = 0; b < 4; b++) {
        bal[b] = __ballot((m >> b) & 1);
        nbal[b] = __ballot(((m >> b) & 1) && nearp);
    }
    const uint64_t wide_bal = __ballot(has && st.wide[t]);
    if (lane == 0)
#pragma unroll
        for (int b = 0; b < 4; b++) {
            st.wcnt[w][b] = (int)__popcll(bal[b]);
            st.ncnt[w][b] = (int)__popcll(nbal[b]);
        }
    if (t < 4) st.wrap[t] = 0;
    __syncthreads();
    // a wide entry reaches every sub-tile (its mask is 0xF)
    if (lane == 0 && wide_bal)
#pragma unroll
        for (int b = 0; b < 4; b++) st.wrap[b] = 1;
#pragma unroll
    for (int b = 0; b < 4; b++) {
        if ((m >> b) & 1) {
            int pos = count_below(bal[b]);
            for (int ww = 0; ww < w; ww++) pos += st.wcnt[ww][b];
            st.list[b][pos] = (unsigned short)t;
        }
    }
    if (t < 4) st.len[t] = st.wcnt[0][t] + st.wcnt[1][t] + st.wcnt[2][t] + st.wcnt[3][t];
    __syncthreads();
}

// exclusive scan over the 256 threads of a workgroup; total = sum of all
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t &total, uint32_t *s_w)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t v = x;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(v, off);
        if (lane >= off) v += y;
    }
    if (lane == 63) s_w[w] = v;
    __syncthreads();
    uint32_t pre = 0;
    for (int i = 0; i < w; i++) pre += s_w[i];
    total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    return pre + v - x;
}

}  // namespace rxgs
