// Backward kernels of librxgs for gfx950 (App. D of RxGS: the backward runs on
// the same (tile, receiver) grid as the forward and accumulates Gaussian-level
// gradients over receivers and directions with atomics).
//
//   k_blend_bwd     reverse walk of each tile list from the last composited
//                   entry: T_before = T_after / (1 - w) from the saved final
//                   transmittance; per entry dL/ds (per receiver) and dL/d(u,
//                   v, conic, opacity) summed over the wave (DPP), one atomic
//                   per wave.                                        [VALU]
//   k_mlp_bwd       persistent FP32-MFMA backward of layers 2 and 3 over the
//                   same work items as the forward (recompute, dz2, dx1 =
//                   W2^T dz2, dW2 = dz2^T x1), per-wave partial sums. [MFMA]
//   k_mlp_*_w1      layer-1 weights (receiver and Gaussian parts), bias and
//                   feature gradients.
//   k_project_bwd   per (view, visible Gaussian): projected-record gradients
//                   to mean, log-scale, quaternion and opacity logit (FP64).
#include "device_common.h"

#include <cmath>

namespace rxgs {

constexpr int MLPB_PART = 4096 + 64 + 128 + 2 + 62;   // dW2, db2, dW3, db3, pad
constexpr int W1B_CHUNK = 128;                        // Gaussians per dW1b partial
constexpr int RED_GROUPS = 64;                        // row groups of the two-stage column sums
constexpr int MLPB_RSUB = 4;                          // receivers per virtual item of the MLP backward (at least)
constexpr float LN2F = 0.69314718055994531f;

// ----------------------------------------------------------------------------
// Same (tile, receiver chunk) grid, pixel mapping, LDS staging and per-wave
// entry lists as the forward; batches are staged from the end of the consumed
// part of the tile list towards its start and walked in reverse.  Each
// forward chunk is split into `split` blocks of at most R receivers.  The
// per-entry wave sums of a batch are accumulated in LDS over the block's four
// waves and flushed to global memory once per batch, one entry per thread:
// global atomics inside the walk stall it (they count against the wave's
// outstanding-memory budget) and contend across the waves of a tile.
// Deterministic variant (DET): each wave adds its entry sums over its 64
// lanes in a fixed order into its own LDS slots, the four waves' slots are
// added in order at the flush, and every (pair, receiver block) gets its own
// partial in global memory (no atomics), stored at the pair's emission slot
// (its position's first slot plus the tile's index in the position's tile
// enumeration), so a later gather adds each position's partials from one
// contiguous range, in emission order.
struct DetPartials {
    float *gP;          // [block of the view][Dpad][8]: (u, v, a, b, c, o) partials per pair, emission slot
    float *dSP;         // [row of the view][Dpad][2]: dL/ds partials per pair, emission slot
    int64_t Dpad;
    const int4 *vinfo;  // per view (first row, rows, visible, -)
    const float4 *sbox; // binning box of each sorted position
    const uint32_t *poff;   // first pair slot of each sorted position within its view
    const uint32_t *pbase;  // first pair slot of each view
};

template <int R, bool DET>
__global__ __launch_bounds__(BLOCK) void k_blend_bwd(
    const float4 *__restrict__ srec, const uint32_t *__restrict__ pval, const uint2 *__restrict__ ranges,
    const float2 *__restrict__ rad, const int4 *__restrict__ chunks, int split, int64_t Kp, DevGrid g,
    int tx_mode, const float *__restrict__ C, const float *__restrict__ dC, const float *__restrict__ dP,
    const float *__restrict__ dA, const float *__restrict__ Tfin, const int *__restrict__ nlast, float *__restrict__ dS,
    float *__restrict__ g2d, uint8_t *__restrict__ live, DetPartials det)
{
    constexpr int NV = 6 + 2 * R;   // values per entry: six record gradients, then (Re, Im) per receiver
    __shared__ BlendStage st;
    __shared__ float2 s_rad[R][BLOCK];
    __shared__ float s_acc[DET ? 1 : 6][BLOCK];
    __shared__ float2 s_dacc[DET ? 1 : R][BLOCK];
    __shared__ float s_accw[DET ? 4 : 1][DET ? NV : 1][BLOCK];
    __shared__ int s_max[4];

    const int tile = blockIdx.x;
    const int4 ch = chunks[blockIdx.y / split];
    const int sub = blockIdx.y - (blockIdx.y / split) * split;
    const int view = ch.x, j0 = ch.y + sub * R, nrx = min(ch.z - sub * R, R);
    if (nrx <= 0) return;   // uniform over the block, before any barrier
    const int tread = tx_mode ? view : j0;
    const int ty = tile / g.tiles_x, tx = tile - ty * g.tiles_x;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int row = ty * TILE + 8 * (wv >> 1) + (lane >> 3), col = tx * TILE + 8 * (wv & 1) + (lane & 7);
    const bool inside = row < g.H && col < g.W;
    const float rowf = (float)row, colf = (float)col;
    const float Wf = (float)g.W, halfW = 0.5f * (float)g.W;
    const uint2 rg = ranges[(size_t)view * g.tiles + tile];
    const int64_t view_end = ((int64_t)view + 1) * Kp;
    const size_t P = (size_t)g.H * g.W;
    const size_t pix = (size_t)row * g.W + col;

    float T = 1.f;
    int last = 0;
    if (inside) {
        T = Tfin[(size_t)tread * P + pix];
        last = nlast[(size_t)tread * P + pix];
    }
    float2 G[R], A[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        G[r] = make_float2(0.f, 0.f);
        A[r] = make_float2(0.f, 0.f);
        if (inside && r < nrx) {
            const size_t j = (size_t)(j0 + r);
            // dL/dC of the pixel: the spectrum's own gradient, the power's
            // (d|C|^2/dC = 2 C) and the amplitude's (d sqrt(|C|^2 + 1e-8)/dC = C / amplitude)
            const float gp = dP ? 2.f * dP[j] : 0.f;
            const float cx = C[(j * 2) * P + pix], cy = C[(j * 2 + 1) * P + pix];
            G[r].x = (dC ? dC[(j * 2) * P + pix] : 0.f) + gp * cx;
            G[r].y = (dC ? dC[(j * 2 + 1) * P + pix] : 0.f) + gp * cy;
            if (dA) {
                const float ga = dA[j * P + pix] / sqrtf(cx * cx + cy * cy + AMP_EPS);
                G[r].x += ga * cx;
                G[r].y += ga * cy;
            }
        }
    }
    int m = last;
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if (lane == 0) s_max[wv] = m;
    __syncthreads();
    const int maxlast = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));

    for (int end = maxlast; end > 0; end -= BLOCK) {
        const int start = max(0, end - BLOCK);
        const int cnt = end - start;
        __syncthreads();
        uint32_t p = 0;
        if constexpr (DET) {
#pragma unroll
            for (int w = 0; w < 4; w++)
#pragma unroll
                for (int c = 0; c < NV; c++) s_accw[w][c][t] = 0.f;
        } else {
#pragma unroll
            for (int c = 0; c < 6; c++) s_acc[c][t] = 0.f;
#pragma unroll
            for (int r = 0; r < R; r++) s_dacc[r][t] = make_float2(0.f, 0.f);
        }
        if (t < cnt) {
            p = (uint32_t)min((int64_t)pval[rg.x + start + t], view_end - 1);
            const int64_t s = max((int64_t)p - (int64_t)view * Kp, (int64_t)0);
#pragma unroll
            for (int r = 0; r < R; r++)
                s_rad[r][t] = (r < nrx) ? rad[(size_t)(j0 + r) * Kp + s] : make_float2(0.f, 0.f);
        }
        stage_batch(st, srec, p, t < cnt, tx, ty, g);
        const int n = st.len[wv];
        for (int i = n - 1; i >= 0; i--) {
            const int e = st.list[wv][i];
            bool act = inside && (start + e) < last;
            float gu = 0.f, gv = 0.f, gca = 0.f, gcb = 0.f, gcc = 0.f, glo = 0.f;
            float2 dsr[R];
#pragma unroll
            for (int r = 0; r < R; r++) dsr[r] = make_float2(0.f, 0.f);
            if (act) {
                const float4 r0 = st.r0[e];
                const float4 r1 = st.r1[e];
                float du = (colf - r0.x) - r0.y;
                if (st.wide[e]) {
                    if (du >= halfW) du -= Wf;
                    else if (du < -halfW) du += Wf;
                }
                const float dv = (rowf - r0.z) - r0.w;
                const float ex = blend_exponent(du, dv, r1);
                const float wr = __builtin_amdgcn_exp2f(ex);
                const float w = fminf(W_MAX, wr);
                if (w >= ALPHA_MIN) {
                    // 1 / (1 - w) by the hardware reciprocal (1 ulp; 1 - w >= 0.01):
                    // over a pixel's few dozen composited entries the recovered
                    // transmittance stays within ~1e-6 of the forward's
                    const float rw = __builtin_amdgcn_rcpf(1.f - w);
                    const float Tb = T * rw;
                    const float tw = Tb * w;
                    float dw = 0.f;
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        const float2 sv = s_rad[r][e];
                        dsr[r] = make_float2(tw * G[r].x, tw * G[r].y);
                        dw += G[r].x * fmaf(T, sv.x, -A[r].x) + G[r].y * fmaf(T, sv.y, -A[r].y);
                        A[r].x = fmaf(tw, sv.x, A[r].x);
                        A[r].y = fmaf(tw, sv.y, A[r].y);
                    }
                    dw *= rw;
                    if (wr < W_MAX) {
                        const float gex = dw * w * LN2F;
                        gu = -gex * (2.f * r1.x * du + r1.y * dv);
                        gv = -gex * (r1.y * du + 2.f * r1.z * dv);
                        gca = gex * du * du;
                        gcb = gex * du * dv;
                        gcc = gex * dv * dv;
                        glo = gex;
                    }
                    T = Tb;
                } else {
                    act = false;
                }
            }
            if (__ballot(act) == 0) continue;   // uniform across the wave
            float vals[6] = {gu, gv, gca, gcb, gcc, glo};
            if constexpr (DET) {
                // the wave's sum: its four 16-lane row sums added in order
                auto wave_total = [&](float x) {
                    const float v = row_sum(x);
                    const int b = __float_as_int(v);
                    return ((__int_as_float(__builtin_amdgcn_readlane(b, 15)) +
                             __int_as_float(__builtin_amdgcn_readlane(b, 31))) +
                            __int_as_float(__builtin_amdgcn_readlane(b, 47))) +
                           __int_as_float(__builtin_amdgcn_readlane(b, 63));
                };
#pragma unroll
                for (int c = 0; c < 6; c++) {
                    const float v = wave_total(vals[c]);
                    if (lane == 0) s_accw[wv][c][e] = v;
                }
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (r < nrx) {
                        const float vx = wave_total(dsr[r].x);
                        const float vy = wave_total(dsr[r].y);
                        if (lane == 0) {
                            s_accw[wv][6 + 2 * r][e] = vx;
                            s_accw[wv][7 + 2 * r][e] = vy;
                        }
                    }
                }
                continue;
            }
            // sums over each 16-lane row, added into the batch's LDS
            // accumulators by the rows' last lanes
            const bool row_last = (lane & 15) == 15;
#pragma unroll
            for (int c = 0; c < 6; c++) {
                const float v = row_sum(vals[c]);
                if (row_last && v != 0.f) atomicAdd(&s_acc[c][e], v);
            }
#pragma unroll
            for (int r = 0; r < R; r++) {
                if (r < nrx) {
                    const float vx = row_sum(dsr[r].x);
                    const float vy = row_sum(dsr[r].y);
                    if (row_last) {
                        if (vx != 0.f) atomicAdd(&s_dacc[r][e].x, vx);
                        if (vy != 0.f) atomicAdd(&s_dacc[r][e].y, vy);
                    }
                }
            }
        }
        __syncthreads();
        if constexpr (DET) {
            // thread t owns entry t: the four waves' sums in order, stored at
            // the entry's pair slot for this block of receivers
            if (t < cnt) {
                const uint32_t pe = st.p[t];
                // the pair's emission slot
                const float4 b = det.sbox[pe];
                int ty0, ty1, a0, a1, b0, b1;
                (void)tile_rows(b.y, b.w, g.H, ty0, ty1);
                (void)tile_cols(b.x, b.z, g.W, g.tiles_x, a0, a1, b0, b1);
                const int64_t d = (int64_t)det.pbase[view] + det.poff[pe] + tile_rank(ty, tx, ty0, a0, a1, b0, b1);
                const int4 vi = det.vinfo[view];
                const int64_t blk = (j0 - vi.x) / R;
                float *gp = det.gP + ((size_t)blk * det.Dpad + d) * 8;
#pragma unroll
                for (int c = 0; c < 6; c++)
                    gp[c] = ((s_accw[0][c][t] + s_accw[1][c][t]) + s_accw[2][c][t]) + s_accw[3][c][t];
                bool any = false;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (r < nrx) {
                        const float vx = ((s_accw[0][6 + 2 * r][t] + s_accw[1][6 + 2 * r][t]) +
                                          s_accw[2][6 + 2 * r][t]) + s_accw[3][6 + 2 * r][t];
                        const float vy = ((s_accw[0][7 + 2 * r][t] + s_accw[1][7 + 2 * r][t]) +
                                          s_accw[2][7 + 2 * r][t]) + s_accw[3][7 + 2 * r][t];
                        float *dd = det.dSP + ((size_t)(j0 + r - vi.x) * det.Dpad + d) * 2;
                        dd[0] = vx;
                        dd[1] = vy;
                        any = any || vx != 0.f || vy != 0.f;
                    }
                }
                if (any) live[pe / MLP_PAIRS] = 1;
            }
            continue;
        }
        // flush the batch: thread t owns entry t
        if (t < cnt) {
            const uint32_t pe = st.p[t];
#pragma unroll
            for (int c = 0; c < 6; c++) {
                const float v = s_acc[c][t];
                if (v != 0.f) atomicAdd(&g2d[(size_t)pe * 8 + c], v);
            }
            const int64_t s = (int64_t)pe - (int64_t)view * Kp;
            bool any = false;
#pragma unroll
            for (int r = 0; r < R; r++) {
                if (r < nrx) {
                    const float2 d = s_dacc[r][t];
                    float *dd = dS + ((size_t)(j0 + r) * Kp + s) * 2;
                    if (d.x != 0.f) atomicAdd(dd, d.x);
                    if (d.y != 0.f) atomicAdd(dd + 1, d.y);
                    any = any || d.x != 0.f || d.y != 0.f;
                }
            }
            // the MLP backward only visits position blocks marked here
            if (any) live[pe / MLP_PAIRS] = 1;
        }
    }
}

// ----------------------------------------------------------------------------
// direct radiance: dL/d radiance_k = sum over receivers of dL/ds at k's positions
__global__ __launch_bounds__(BLOCK) void k_rad_direct_bwd(const float2 *__restrict__ dS,
                                                          const uint32_t *__restrict__ order,
                                                          const unsigned long long *__restrict__ counters,
                                                          const int *__restrict__ rxview, int N, int64_t Kp,
                                                          int64_t K, float *__restrict__ grad)
{
    const int64_t idx = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= (int64_t)N * Kp) return;
    const int64_t j = idx / Kp, s = idx - j * Kp;
    const int v = rxview[j];
    if (s >= (int64_t)counters[2 * (size_t)v]) return;
    const float2 d = dS[idx];
    if (d.x == 0.f && d.y == 0.f) return;
    const int64_t k = min((int64_t)order[(size_t)v * Kp + s], K - 1);
    atomicAdd(&grad[2 * k], d.x);
    atomicAdd(&grad[2 * k + 1], d.y);
}

// Live virtual items of the MLP backward, listed in index order (a virtual
// item is live when its receiver range is not empty and its position block
// holds a nonzero dL/ds).  The MLP backward then gives the item of rank r to
// wave r mod (waves): the few hundred live items of an RX training step get
// a wave each, whatever their positions in the item list.  Two launches over
// chunks of 1024 virtual items: counts per chunk, then each chunk writes its
// live items after those of the chunks before it.
__device__ __forceinline__ bool mlp_virt_live(int x, const int4 *__restrict__ items, int n1,
                                              const int4 *__restrict__ items2, int nsub, int rsub, int64_t Kp,
                                              const uint8_t *__restrict__ live)
{
    const int ii = x / nsub;
    const int4 it = ii < n1 ? items[ii] : items2[ii - n1];
    return (x % nsub) * rsub < (it.w & 255) && live[((size_t)it.x * Kp + it.y) / MLP_PAIRS] != 0;
}

template <bool WRITE>
__global__ __launch_bounds__(BLOCK) void k_live_list(const int4 *__restrict__ items, int n1,
                                                     const int4 *__restrict__ items2, const int *__restrict__ count2,
                                                     int nsub, int64_t Kp, const uint8_t *__restrict__ live,
                                                     uint32_t *__restrict__ counts, uint32_t *__restrict__ nlist,
                                                     uint32_t *__restrict__ list)
{
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x;
    const int nvirt = (n1 + (items2 ? *count2 : 0)) * nsub, rsub = (MLP_RG + nsub - 1) / nsub;
    const int x0 = (int)blockIdx.x * 4 * BLOCK + 4 * t;
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (x0 + j < nvirt && mlp_virt_live(x0 + j, items, n1, items2, nsub, rsub, Kp, live)) m |= 1u << j;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan((uint32_t)__builtin_popcount(m), tot, s_w);
    if (!WRITE) {
        if (t == 0) counts[blockIdx.x] = tot;
        return;
    }
    uint32_t pre = 0;
    for (uint32_t g = t; g < blockIdx.x; g += BLOCK) pre += counts[g];
    uint32_t before;
    (void)block_exclusive_scan(pre, before, s_w);
    uint32_t pos = before + ex;
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (m & (1u << j)) list[pos++] = (uint32_t)(x0 + j);
    if (blockIdx.x == gridDim.x - 1 && t == 0) *nlist = before + tot;
}

// ----------------------------------------------------------------------------
// MLP backward, layers 2 and 3, persistent waves.  Per work item (view, 32
// sorted positions, receivers) and receiver:
//   x1 = relu(L_k + G_j)                     lane = pair, hid_of order
//   z2 = b2 + W2 x1          (MFMA, A = w2a)   lane = pair
//   dz2 = (W3^T ds) * [z2 > 0]
//   dx1 = (W2^T dz2) * [x1 > 0]  (MFMA, A = w2b, B = dz2 registers)
//   dL_k += dx1 (registers), dG_j += sum over pairs of dx1 (DPP, atomics)
//   z2 transposed through LDS to lane = hidden unit, then
//   dW2 += dz2^T x1 over the 32 pairs (MFMA), db2, dW3, db3 (VALU)
// Deterministic variant: each live position block has a slot (its rank);
// the Gaussian term of an item is stored per (slot, receiver group, pair),
// the receiver term per (slot, row of the view), for fixed-order gathers.
struct DetMlp {
    float *dLv;          // [slot][receiver group][32][64]
    float *dGp;          // [slot][row of the view][64]
    const int *rank;     // per position block: slot or -1
    const int4 *vinfo;   // per view (first row, rows, visible, -)
    int nrg_max, rows_max;
};

template <bool DET>
__global__ __launch_bounds__(BLOCK) void k_mlp_bwd(
    const float *__restrict__ Lp, const float *__restrict__ Gp, const float *__restrict__ w2a,
    const float *__restrict__ w2b, const float4 *__restrict__ tab, const float *__restrict__ W3,
    const uint32_t *__restrict__ order, const int4 *__restrict__ items, int nitems,
    const int4 *__restrict__ items2, const int *__restrict__ count2, int nsub, int64_t Kp,
    int64_t K, const uint8_t *__restrict__ live, const uint32_t *__restrict__ list, const uint32_t *__restrict__ nlist,
    const float2 *__restrict__ dS, float *__restrict__ dL, float *__restrict__ dG, float *__restrict__ part,
    DetMlp det)
{
    __shared__ float s_w2a[2 * 32 * 64];
    __shared__ float s_w2b[2 * 32 * 64];
    __shared__ float4 s_tab[64];
    __shared__ float s_z2[4][32][65];
    __shared__ float2 s_ds[4][32];
    for (int i = threadIdx.x; i < 2 * 32 * 64; i += BLOCK) {
        s_w2a[i] = w2a[i];
        s_w2b[i] = w2b[i];
    }
    if (threadIdx.x < 64) s_tab[threadIdx.x] = tab[threadIdx.x];
    __syncthreads();

    const int lane = threadIdx.x & 63, h = lane >> 5, pl = lane & 31, wv = threadIdx.x >> 6;
    const int gw = blockIdx.x * (BLOCK / 64) + wv, nw = gridDim.x * (BLOCK / 64);
    floatx16 dw2[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) dw2[a][b][r] = 0.f;
    float db2a[2] = {0.f, 0.f}, dw3a[2][2] = {{0.f, 0.f}, {0.f, 0.f}}, db3a[2] = {0.f, 0.f};
    float w3o[2][2];
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int ob = 0; ob < 2; ob++) w3o[c][ob] = W3[c * HID + pl + 32 * ob];
    const int pos_i0 = hid_pos(pl), pos_i1 = hid_pos(pl + 32);

    // A pair whose dL/ds is zero for every receiver adds exactly zero to every
    // gradient below.  In optically thick scenes only the nearest few hundred
    // Gaussians of a view are composited, so most items have no nonzero dL/ds;
    // the blend backward marks the position blocks that do, and each round
    // reads the marks of this wave's next 64 items at once.
    // Each work item is split into nsub virtual items of at most
    // MLP_RG / nsub receivers, so a live item's receivers spread over waves
    // instead of running one after another in one wave (nsub = 1 when every
    // view has few receivers, as in RX mode).
    // work items: the forward's list, then (a radiance-prefix forward) the
    // list of its blocks past the prefix that hold composited entries
    const int n1 = nitems;
    nitems += items2 ? *count2 : 0;
    const int nvirt = nitems * nsub, rsub = (MLP_RG + nsub - 1) / nsub;
    // Virtual items are dealt to waves in a scattered order, x -> x * HASH mod
    // nvirt (a bijection: HASH is a prime above any count), so the few live
    // items at the start of every view spread over waves instead of piling
    // onto the same ones when the views' item counts are regular.
    // With the list of live virtual items, the item of rank r goes to wave
    // r mod (waves) instead.
    constexpr uint64_t HASH = 2654435761ull;
    const int nsrc = list ? (int)*nlist : nvirt;
    for (int base = gw; base < nsrc; base += 64 * nw) {
    uint64_t todo;
    {
        const int mine = base + lane * nw;
        bool lv = false;
        if (mine < nsrc && list) {
            lv = true;
        } else if (mine < nsrc) {
            const int vm = (int)(((uint64_t)mine * HASH) % (uint64_t)nvirt);
            const int ii = vm / nsub;
            const int4 it = ii < n1 ? items[ii] : items2[ii - n1];
            const int sub = vm % nsub;
            lv = sub * rsub < (it.w & 255) && live[((size_t)it.x * Kp + it.y) / MLP_PAIRS] != 0;
        }
        todo = __ballot(lv);
    }
    while (todo) {
        const int src = base + __builtin_ctzll(todo) * nw;
        const int vitem = list ? (int)list[src] : (int)(((uint64_t)src * HASH) % (uint64_t)nvirt);
        todo &= todo - 1;
        const int iv = vitem / nsub;
        const int4 it = iv < n1 ? items[iv] : items2[iv - n1];
        const int sub = vitem % nsub;
        const int view = it.x, s0 = it.y, j0 = it.z + sub * rsub;
        const int nj = min(rsub, (it.w & 255) - sub * rsub);
        const int64_t s = s0 + pl;
        const int nvalid = it.w >> 8;
        const bool valid = pl < nvalid;
        const int64_t nv = (int64_t)s0 + nvalid;
        const size_t obase = (size_t)view * Kp;
        const uint32_t k = (uint32_t)min((int64_t)order[obase + (valid ? s : s0)], K - 1);
        float l[32];
        {
            const float4 *src = reinterpret_cast<const float4 *>(Lp + (size_t)k * HID + h * 32);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const float4 x = src[q];
                l[4 * q] = x.x; l[4 * q + 1] = x.y; l[4 * q + 2] = x.z; l[4 * q + 3] = x.w;
            }
        }
        // Gaussians of the pairs 2 t + h, for the lane = hidden-unit layout
        float lt0[16], lt1[16];
#pragma unroll
        for (int tt = 0; tt < 16; tt++) {
            const int64_t sp = min((int64_t)(s0 + 2 * tt + h), nv - 1);
            const uint32_t kp = (uint32_t)min((int64_t)order[obase + sp], K - 1);
            lt0[tt] = Lp[(size_t)kp * HID + pos_i0];
            lt1[tt] = Lp[(size_t)kp * HID + pos_i1];
        }
        float dl[32];
#pragma unroll
        for (int q = 0; q < 32; q++) dl[q] = 0.f;

        for (int jj = 0; jj < nj; jj++) {
            const int j = j0 + jj;
            const float2 dsv = valid ? dS[(size_t)j * Kp + s] : make_float2(0.f, 0.f);
            if (__ballot(dsv.x != 0.f || dsv.y != 0.f) == 0) continue;   // adds exactly zero
            float x1[32];
            {
                const float4 *gs = reinterpret_cast<const float4 *>(Gp + (size_t)j * HID + h * 32);
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const float4 gv = gs[q];
                    x1[4 * q] = fmaxf(l[4 * q] + gv.x, 0.f);
                    x1[4 * q + 1] = fmaxf(l[4 * q + 1] + gv.y, 0.f);
                    x1[4 * q + 2] = fmaxf(l[4 * q + 2] + gv.z, 0.f);
                    x1[4 * q + 3] = fmaxf(l[4 * q + 3] + gv.w, 0.f);
                }
            }
            floatx16 a0, a1;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                a0[r] = s_tab[(h * 2 + 0) * 16 + r].z;
                a1[r] = s_tab[(h * 2 + 1) * 16 + r].z;
            }
#pragma unroll
            for (int tt = 0; tt < 32; tt++) {
                a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(s_w2a[(0 * 32 + tt) * 64 + lane], x1[tt], a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f32_32x32x2f32(s_w2a[(1 * 32 + tt) * 64 + lane], x1[tt], a1, 0, 0, 0);
            }
            float dz[32];
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const float4 ta = s_tab[(h * 2 + 0) * 16 + r];
                const float4 tb = s_tab[(h * 2 + 1) * 16 + r];
                dz[r] = a0[r] > 0.f ? ta.x * dsv.x + ta.y * dsv.y : 0.f;
                dz[16 + r] = a1[r] > 0.f ? tb.x * dsv.x + tb.y * dsv.y : 0.f;
                s_z2[wv][pl][hid_of(h, r)] = a0[r];
                s_z2[wv][pl][hid_of(h, 16 + r)] = a1[r];
            }
            if (h == 0) s_ds[wv][pl] = dsv;
            floatx16 c0, c1;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                c0[r] = 0.f;
                c1[r] = 0.f;
            }
#pragma unroll
            for (int tt = 0; tt < 32; tt++) {
                c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(s_w2b[(0 * 32 + tt) * 64 + lane], dz[tt], c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(s_w2b[(1 * 32 + tt) * 64 + lane], dz[tt], c1, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const float d0 = x1[r] > 0.f ? c0[r] : 0.f;
                const float d1 = x1[16 + r] > 0.f ? c1[r] : 0.f;
                dl[r] += d0;
                dl[16 + r] += d1;
                const float s0v = half_wave_sum(d0);
                const float s1v = half_wave_sum(d1);
                if (pl == 31) {
                    if constexpr (DET) {
                        const int rk = det.rank[((size_t)view * Kp + s0) / MLP_PAIRS];
                        float *dg = det.dGp + ((size_t)rk * det.rows_max + (j - det.vinfo[view].x)) * HID + h * 32;
                        dg[r] = s0v;
                        dg[16 + r] = s1v;
                    } else {
                        if (s0v != 0.f) atomicAdd(&dG[(size_t)j * HID + h * 32 + r], s0v);
                        if (s1v != 0.f) atomicAdd(&dG[(size_t)j * HID + h * 32 + 16 + r], s1v);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            const float g_i0 = Gp[(size_t)j * HID + pos_i0], g_i1 = Gp[(size_t)j * HID + pos_i1];
#pragma unroll
            for (int tt = 0; tt < 16; tt++) {
                const int pr = 2 * tt + h;
                const float2 d = s_ds[wv][pr];
                const float z0 = s_z2[wv][pr][pl], z1 = s_z2[wv][pr][pl + 32];
                const float m0 = z0 > 0.f ? 1.f : 0.f, m1 = z1 > 0.f ? 1.f : 0.f;
                const float dzt0 = m0 * (w3o[0][0] * d.x + w3o[1][0] * d.y);
                const float dzt1 = m1 * (w3o[0][1] * d.x + w3o[1][1] * d.y);
                db2a[0] += dzt0;
                db2a[1] += dzt1;
                dw3a[0][0] = fmaf(d.x, m0 * z0, dw3a[0][0]);
                dw3a[1][0] = fmaf(d.y, m0 * z0, dw3a[1][0]);
                dw3a[0][1] = fmaf(d.x, m1 * z1, dw3a[0][1]);
                dw3a[1][1] = fmaf(d.y, m1 * z1, dw3a[1][1]);
                const float xb0 = fmaxf(lt0[tt] + g_i0, 0.f), xb1 = fmaxf(lt1[tt] + g_i1, 0.f);
                dw2[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(dzt0, xb0, dw2[0][0], 0, 0, 0);
                dw2[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(dzt0, xb1, dw2[0][1], 0, 0, 0);
                dw2[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(dzt1, xb0, dw2[1][0], 0, 0, 0);
                dw2[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(dzt1, xb1, dw2[1][1], 0, 0, 0);
            }
            if (lane == 0)
                for (int q = 0; q < 32; q++) {
                    db3a[0] += s_ds[wv][q].x;
                    db3a[1] += s_ds[wv][q].y;
                }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        if constexpr (DET) {
            const int rk = det.rank[((size_t)view * Kp + s0) / MLP_PAIRS];
            const int a = (j0 - det.vinfo[view].x) / MLP_RG;
            float *dl_out = det.dLv + (((size_t)rk * det.nrg_max + a) * MLP_PAIRS + pl) * HID + h * 32;
#pragma unroll
            for (int q = 0; q < 32; q++) dl_out[q] = dl[q];
        } else if (valid) {
#pragma unroll
            for (int q = 0; q < 32; q++)
                if (dl[q] != 0.f) atomicAdd(&dL[(size_t)k * HID + h * 32 + q], dl[q]);
        }
    }
    }
    // per-wave partial sums (natural layouts), reduced in a fixed order later
    float *pw = part + (size_t)gw * MLPB_PART;
#pragma unroll
    for (int ob = 0; ob < 2; ob++)
#pragma unroll
        for (int ib = 0; ib < 2; ib++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int o = 32 * ob + 8 * (r >> 2) + 4 * h + (r & 3);
                const int i = 32 * ib + pl;
                pw[o * HID + i] = dw2[ob][ib][r];
            }
#pragma unroll
    for (int ob = 0; ob < 2; ob++) {
        const float b = db2a[ob] + __shfl_xor(db2a[ob], 32);
        const float w0 = dw3a[0][ob] + __shfl_xor(dw3a[0][ob], 32);
        const float w1 = dw3a[1][ob] + __shfl_xor(dw3a[1][ob], 32);
        if (h == 0) {
            pw[4096 + pl + 32 * ob] = b;
            pw[4096 + 64 + pl + 32 * ob] = w0;
            pw[4096 + 64 + 64 + pl + 32 * ob] = w1;
        }
    }
    if (lane == 0) {
        pw[4096 + 192] = db3a[0];
        pw[4096 + 193] = db3a[1];
    }
}

// First stage of a fixed-order column sum of a (nrows x ld) partial-sum
// matrix: group blockIdx.y sums its contiguous run of rows in order, in FP64.
// The groups run in parallel; the second stage adds the RED_GROUPS group sums
// in order, so the result does not depend on scheduling.
__global__ __launch_bounds__(BLOCK) void k_colsum_groups(const float *__restrict__ part, int nrows, int ld, int ncols,
                                                         double *__restrict__ out)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= ncols) return;
    const int per = (nrows + RED_GROUPS - 1) / RED_GROUPS;
    const int r0 = blockIdx.y * per, r1 = min(nrows, r0 + per);
    double acc = 0.0;
#pragma unroll 8
    for (int r = r0; r < r1; r++) acc += part[(size_t)r * ld + c];
    out[(size_t)blockIdx.y * ncols + c] = acc;
}

// second stage: the flat MLP gradient of layers 2 and 3 from the group sums
__global__ __launch_bounds__(BLOCK) void k_mlp_bwd_reduce(const double *__restrict__ red, float *__restrict__ gmlp)
{
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= 4096 + 194) return;
    double acc = 0.0;
    for (int gi = 0; gi < RED_GROUPS; gi++) acc += red[(size_t)gi * (4096 + 194) + e];
    const int W2OFF = HID * MLP_IN + HID, B2OFF = W2OFF + HID * HID, W3OFF = B2OFF + HID, B3OFF = W3OFF + 2 * HID;
    int dst;
    if (e < 4096) dst = W2OFF + e;
    else if (e < 4096 + 64) dst = B2OFF + (e - 4096);
    else if (e < 4096 + 192) dst = W3OFF + (e - 4096 - 64);
    else dst = B3OFF + (e - 4096 - 192);
    gmlp[dst] = (float)acc;
}

// layer 1, receiver part and bias: dW1[:, :36] = sum_j dG_j gamma(r_j)^T, db1 = sum_j dG_j
__global__ __launch_bounds__(BLOCK) void k_mlp_w1a(const float *__restrict__ dG, const float *__restrict__ rx, int N,
                                                   float *__restrict__ gmlp)
{
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= HID * (ENC + 1)) return;
    const int d = idx / (ENC + 1), e = idx % (ENC + 1);
    const int pos = hid_pos(d);
    double acc = 0.0;
    if (e == ENC) {
        for (int j = 0; j < N; j++) acc += dG[(size_t)j * HID + pos];
        gmlp[HID * MLP_IN + d] = (float)acc;
        return;
    }
    const int a = e / 12, f = (e % 12) / 2, cs = e & 1;
    for (int j = 0; j < N; j++) {
        float sn, cn;
        sincosf(ldexpf(rx[3 * j + a], f), &sn, &cn);
        acc += (double)dG[(size_t)j * HID + pos] * (double)(cs ? cn : sn);
    }
    gmlp[d * MLP_IN + e] = (float)acc;
}

// layer 1, Gaussian part: partial sums of dL_k f_k^T over chunks of Gaussians
__global__ __launch_bounds__(BLOCK) void k_mlp_w1b_part(const float *__restrict__ dL, const float *__restrict__ feat,
                                                        int64_t K, float *__restrict__ part)
{
    __shared__ float s_dl[W1B_CHUNK][HID + 1];
    __shared__ float s_f[W1B_CHUNK][FEAT + 1];
    const int64_t k0 = (int64_t)blockIdx.x * W1B_CHUNK;
    const int n = (int)min((int64_t)W1B_CHUNK, K - k0);
    for (int i = threadIdx.x; i < W1B_CHUNK * HID; i += BLOCK) {
        const int kk = i / HID, d = i % HID;
        s_dl[kk][d] = kk < n ? dL[(size_t)(k0 + kk) * HID + hid_pos(d)] : 0.f;
    }
    __syncthreads();
    // rows with a zero dL add exactly zero: list the others in increasing
    // order (threads 0..127 own one row each; waves 0 and 1 hold them)
    __shared__ unsigned char s_list[W1B_CHUNK];
    __shared__ int s_cnt[2];
    bool nz = false;
    if (threadIdx.x < W1B_CHUNK)
        for (int d = 0; d < HID; d++) nz = nz || s_dl[threadIdx.x][d] != 0.f;
    const uint64_t bal = __ballot(nz);
    if ((threadIdx.x & 63) == 0 && threadIdx.x < W1B_CHUNK) s_cnt[threadIdx.x >> 6] = (int)__popcll(bal);
    __syncthreads();
    if (nz) s_list[(threadIdx.x >= 64 ? s_cnt[0] : 0) + count_below(bal)] = (unsigned char)threadIdx.x;
    const int nl = s_cnt[0] + s_cnt[1];
    for (int i = threadIdx.x; i < W1B_CHUNK * FEAT; i += BLOCK) {
        const int kk = i / FEAT, c = i % FEAT;
        s_f[kk][c] = kk < n ? feat[(size_t)(k0 + kk) * FEAT + c] : 0.f;
    }
    __syncthreads();
    // 2048 outputs (64 x 32), 8 per thread
    for (int o = threadIdx.x; o < HID * FEAT; o += BLOCK) {
        const int d = o / FEAT, c = o % FEAT;
        float acc = 0.f;
        for (int q = 0; q < nl; q++) {
            const int kk = s_list[q];
            acc = fmaf(s_dl[kk][d], s_f[kk][c], acc);
        }
        part[(size_t)blockIdx.x * HID * FEAT + o] = acc;
    }
}

__global__ __launch_bounds__(BLOCK) void k_mlp_w1b_reduce(const double *__restrict__ red, float *__restrict__ gmlp)
{
    const int o = blockIdx.x * BLOCK + threadIdx.x;
    if (o >= HID * FEAT) return;
    double acc = 0.0;
    for (int gi = 0; gi < RED_GROUPS; gi++) acc += red[(size_t)gi * HID * FEAT + o];
    const int d = o / FEAT, c = o % FEAT;
    gmlp[d * MLP_IN + ENC + c] = (float)acc;
}

// feature gradients: df_k = W1[:, 36:]^T dL_k, DF_CHUNK Gaussians per block;
// W1's feature columns and 8 dL rows at a time are staged in LDS
constexpr int DF_CHUNK = 64;
__global__ __launch_bounds__(BLOCK) void k_mlp_dfeat(const float *__restrict__ dL, const float *__restrict__ W1,
                                                     int64_t K, float *__restrict__ gfeat)
{
    __shared__ float s_w[HID][FEAT];
    __shared__ float s_dl[8][HID];
    __shared__ int s_nz[8];
    for (int i = threadIdx.x; i < HID * FEAT; i += BLOCK) s_w[i / FEAT][i % FEAT] = W1[(i / FEAT) * MLP_IN + ENC + i % FEAT];
    const int64_t k0 = (int64_t)blockIdx.x * DF_CHUNK;
    const int kk = threadIdx.x >> 5, c = threadIdx.x & 31;
    for (int r = 0; r < DF_CHUNK / 8; r++) {
        const int64_t kb = k0 + 8 * r;
        __syncthreads();
        if (threadIdx.x < 8) s_nz[threadIdx.x] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < 8 * HID; i += BLOCK) {
            const int q = i / HID, d = i % HID;
            const float x = kb + q < K ? dL[(size_t)(kb + q) * HID + hid_pos(d)] : 0.f;
            s_dl[q][d] = x;
            if (x != 0.f) s_nz[q] = 1;
        }
        __syncthreads();
        const int64_t k = kb + kk;
        if (k < K) {
            float acc = 0.f;
            if (s_nz[kk])   // a zero row gives exactly zero
                for (int d = 0; d < HID; d++) acc = fmaf(s_w[d][c], s_dl[kk][d], acc);
            gfeat[(size_t)k * FEAT + c] = acc;
        }
    }
}

// ----------------------------------------------------------------------------
// projection backward (FP64), one thread per (view, visible sorted position)
struct d3 {
    double v, x, y, z;
};
__device__ __forceinline__ d3 D3(double v, double x, double y, double z) { return {v, x, y, z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return {a.v + b.v, a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return {a.v - b.v, a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 operator*(d3 a, d3 b)
{
    return {a.v * b.v, a.x * b.v + a.v * b.x, a.y * b.v + a.v * b.y, a.z * b.v + a.v * b.z};
}
__device__ __forceinline__ d3 operator*(d3 a, double s) { return {a.v * s, a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ d3 operator-(d3 a) { return {-a.v, -a.x, -a.y, -a.z}; }
__device__ __forceinline__ d3 inv(d3 a)
{
    const double r = 1.0 / a.v, r2 = -r * r;
    return {r, a.x * r2, a.y * r2, a.z * r2};
}
__device__ __forceinline__ d3 dsqrt3(d3 a)
{
    const double s = sqrt(a.v), k = 0.5 / s;
    return {s, a.x * k, a.y * k, a.z * k};
}

// The projection backward in three parts, all in FP64: the terms of a
// Gaussian that every view shares (gauss_terms), what one (view, Gaussian)
// record passes back (view_grad), and the rest of the chain from the
// covariance and opacity to the log-scales, raw quaternion and opacity logit
// (cov_grad).  The last part is linear in its inputs for a fixed Gaussian, so
// the views' terms are summed first and it runs once per Gaussian.
// per-Gaussian terms read by every view: covariance upper triangle (00, 01,
// 02, 11, 12, 22) and the mean
struct __align__(16) ProjTerm {
    double S[6];
    float4 pos;
};
static_assert(sizeof(ProjTerm) == PROJ_TERM_BYTES, "ProjTerm layout");

struct GaussTerms {
    double R[3][3], s2[3], S[3][3];
    double w, x, y, z, qn, o;
};

// rotation of the normalised quaternion, squared scales, S = R diag(s2) R^T,
// opacity
__device__ GaussTerms gauss_terms(const float *__restrict__ soa, int64_t K, int64_t k)
{
    GaussTerms t;
    for (int a = 0; a < 3; a++) t.s2[a] = exp(2.0 * (double)soa[(3 + a) * K + k]);
    const double q0 = soa[6 * K + k], q1 = soa[7 * K + k], q2 = soa[8 * K + k], q3 = soa[9 * K + k];
    t.qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const double w = q0 / t.qn, x = q1 / t.qn, y = q2 / t.qn, z = q3 / t.qn;
    t.w = w, t.x = x, t.y = y, t.z = z;
    t.R[0][0] = 1.0 - 2.0 * (y * y + z * z); t.R[0][1] = 2.0 * (x * y - w * z); t.R[0][2] = 2.0 * (x * z + w * y);
    t.R[1][0] = 2.0 * (x * y + w * z); t.R[1][1] = 1.0 - 2.0 * (x * x + z * z); t.R[1][2] = 2.0 * (y * z - w * x);
    t.R[2][0] = 2.0 * (x * z - w * y); t.R[2][1] = 2.0 * (y * z + w * x); t.R[2][2] = 1.0 - 2.0 * (x * x + y * y);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            t.S[a][b] = t.R[a][0] * t.s2[0] * t.R[b][0] + t.R[a][1] * t.s2[1] * t.R[b][1] +
                        t.R[a][2] * t.s2[2] * t.R[b][2];
    t.o = 1.0 / (1.0 + exp(-(double)soa[10 * K + k]));
    return t;
}

// What one (view, Gaussian) record passes back, from its 2-D gradients gg (u,
// v, and the parameters of the blend exponent): to the mean (gp), to the
// covariance as Gs = dL/dS + (dL/dS)^T (entries 00, 01, 02, 11, 12, 22), and
// to the exponent's log2-opacity term (glo).
struct ViewGrad {
    double gp[3], Gs[6], glo;
};

__device__ ViewGrad view_grad(double px, double py, double pz, const double (&S)[3][3],
                              const float *__restrict__ centres, int64_t v, const DevGrid &g,
                              const float *__restrict__ gg)
{
    const double g_u = gg[0], g_v = gg[1], g_ca = gg[2], g_cb = gg[3], g_cc = gg[4];
    const double cx = centres[3 * v], cy = centres[3 * v + 1], cz = centres[3 * v + 2];
    const d3 dx = D3(px - cx, 1, 0, 0), dy = D3(py - cy, 0, 1, 0), dz = D3(pz - cz, 0, 0, 1);
    d3 hh = dx * dx + dy * dy;
    d3 h = dsqrt3(hh);
    if (!(h.v >= H_MIN)) {
        h = D3(H_MIN, 0, 0, 0);
        hh = h * h;
    }
    const d3 rh2 = hh + dz * dz;
    const d3 ihh = inv(hh), irh2h = inv(rh2 * h);
    const double idaz = 1.0 / g.daz, idel = 1.0 / g.del;
    d3 mu[3], mv[3];
    mu[0] = (-dy) * ihh * idaz;
    mu[1] = dx * ihh * idaz;
    mu[2] = D3(0, 0, 0, 0);
    mv[0] = (-(dx * dz)) * irh2h * idel;
    mv[1] = (-(dy * dz)) * irh2h * idel;
    mv[2] = h * inv(rh2) * idel;
    double Smu[3], Smv[3];
    for (int a = 0; a < 3; a++) {
        Smu[a] = S[a][0] * mu[0].v + S[a][1] * mu[1].v + S[a][2] * mu[2].v;
        Smv[a] = S[a][0] * mv[0].v + S[a][1] * mv[1].v + S[a][2] * mv[2].v;
    }
    const double A = mu[0].v * Smu[0] + mu[1].v * Smu[1] + DILATE;
    const double B = mu[0].v * Smv[0] + mu[1].v * Smv[1] + mu[2].v * Smv[2];
    const double Cc = mv[0].v * Smv[0] + mv[1].v * Smv[1] + mv[2].v * Smv[2] + DILATE;
    const double det = A * Cc - B * B, id2 = 1.0 / (det * det);

    // record parameters (ca, cb, cc) -> conic (a, b, c)
    constexpr double L2E = 1.4426950408889634;
    const double g_a = -0.5 * L2E * g_ca, g_b = -L2E * g_cb, g_c = -0.5 * L2E * g_cc;
    // conic = inverse of [[A, B], [B, Cc]]
    const double g_A = (-Cc * Cc * g_a + B * Cc * g_b - B * B * g_c) * id2;
    const double g_B = (2.0 * B * Cc * g_a - (A * Cc + B * B) * g_b + 2.0 * A * B * g_c) * id2;
    const double g_C = (-B * B * g_a + A * B * g_b - A * A * g_c) * id2;
    // Jacobian rows
    double g_mu[3], g_mv[3];
    for (int a = 0; a < 3; a++) {
        g_mu[a] = 2.0 * g_A * Smu[a] + g_B * Smv[a];
        g_mv[a] = 2.0 * g_C * Smv[a] + g_B * Smu[a];
    }
    ViewGrad out;
    for (int a = 0; a < 3; a++) out.gp[a] = 0.0;
    for (int a = 0; a < 3; a++) {
        const double wu = g_mu[a], wvv = g_mv[a];
        out.gp[0] += wu * mu[a].x + wvv * mv[a].x;
        out.gp[1] += wu * mu[a].y + wvv * mv[a].y;
        out.gp[2] += wu * mu[a].z + wvv * mv[a].z;
    }
    for (int a = 0; a < 3; a++) out.gp[a] += g_u * mu[a].v + g_v * mv[a].v;
    // dL/dS = g_A mu mu^T + g_B mu mv^T + g_C mv mv^T, plus its transpose
    int e = 0;
    for (int a = 0; a < 3; a++)
        for (int b = a; b < 3; b++)
            out.Gs[e++] = 2.0 * g_A * mu[a].v * mu[b].v + g_B * (mu[a].v * mv[b].v + mu[b].v * mv[a].v) +
                          2.0 * g_C * mv[a].v * mv[b].v;
    out.glo = gg[5];
    return out;
}

struct CovGrad {
    double gls[3], gq[4], glogit;
};

// from a Gaussian's (summed) Gs and glo: S = R diag(s2) R^T back to the
// log-scales and the raw quaternion, the log2-opacity term back to the logit
__device__ CovGrad cov_grad(const GaussTerms &t, const double (&G6)[6], double glo)
{
    const double Gs[3][3] = {{G6[0], G6[1], G6[2]}, {G6[1], G6[3], G6[4]}, {G6[2], G6[4], G6[5]}};
    const double(&R)[3][3] = t.R;
    const double w = t.w, x = t.x, y = t.y, z = t.z;
    double gR[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0.0;
            for (int c = 0; c < 3; c++) acc += Gs[a][c] * R[c][b];
            gR[a][b] = acc * t.s2[b];
        }
    CovGrad out;
    for (int b = 0; b < 3; b++) {
        double acc = 0.0;
        for (int a = 0; a < 3; a++)
            for (int c = 0; c < 3; c++) acc += R[a][b] * Gs[a][c] * R[c][b];
        out.gls[b] = acc * t.s2[b];   // d s2 / d log-scale = 2 s2; Gs holds dL/dS twice
    }
    // rotation from the normalised quaternion (w, x, y, z)
    const double gw = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
    const double gx = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] - w * gR[1][2] +
                             z * gR[2][0] + w * gR[2][1] - 2.0 * x * gR[2][2]);
    const double gy = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] -
                             w * gR[2][0] + z * gR[2][1] - 2.0 * y * gR[2][2]);
    const double gz = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.0 * z * gR[1][1] +
                             y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
    const double dotq = w * gw + x * gx + y * gy + z * gz;
    out.gq[0] = (gw - w * dotq) / t.qn;
    out.gq[1] = (gx - x * dotq) / t.qn;
    out.gq[2] = (gy - y * dotq) / t.qn;
    out.gq[3] = (gz - z * dotq) / t.qn;
    // log2 o = log2(sigmoid(logit)): d/dlogit = (1 - o) / ln 2
    out.glogit = glo * (1.0 - t.o) / 0.69314718055994531;
    return out;
}

__device__ __forceinline__ bool g2d_zero(const float *gg)
{
    return gg[0] == 0.f && gg[1] == 0.f && gg[2] == 0.f && gg[3] == 0.f && gg[4] == 0.f && gg[5] == 0.f;
}

// per Gaussian: its mean and covariance (upper triangle), read by every view
__global__ __launch_bounds__(BLOCK) void k_proj_terms(const float *__restrict__ soa, int64_t K,
                                                      ProjTerm *__restrict__ pt)
{
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= K) return;
    const GaussTerms t = gauss_terms(soa, K, k);
    ProjTerm p;
    p.S[0] = t.S[0][0], p.S[1] = t.S[0][1], p.S[2] = t.S[0][2];
    p.S[3] = t.S[1][1], p.S[4] = t.S[1][2], p.S[5] = t.S[2][2];
    p.pos = make_float4(soa[k], soa[K + k], soa[2 * K + k], 0.f);
    pt[k] = p;
}

// per (view, visible Gaussian); float atomics add the views' terms: mean
// gradients to their output, Gs and glo per Gaussian (pacc, PACC_STRIDE
// floats each) for k_project_fin
__global__ __launch_bounds__(BLOCK) void k_project_bwd(
    const ProjTerm *__restrict__ pt, int64_t K, int64_t Kp, const float *__restrict__ centres, int V, DevGrid g,
    const uint32_t *__restrict__ order, const unsigned long long *__restrict__ counters,
    const float *__restrict__ g2d, float *__restrict__ gmeans, float *__restrict__ pacc)
{
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= (int64_t)V * Kp) return;
    const int64_t v = p / Kp, s = p - v * Kp;
    if (s >= (int64_t)counters[2 * (size_t)v]) return;
    const float *gg = g2d + (size_t)p * 8;
    if (g2d_zero(gg)) return;
    const int64_t k = min((int64_t)order[p], K - 1);
    const ProjTerm q = pt[k];
    const double S[3][3] = {{q.S[0], q.S[1], q.S[2]}, {q.S[1], q.S[3], q.S[4]}, {q.S[2], q.S[4], q.S[5]}};
    const ViewGrad r = view_grad(q.pos.x, q.pos.y, q.pos.z, S, centres, v, g, gg);
    if (gmeans)
        for (int a = 0; a < 3; a++) atomicAdd(&gmeans[3 * k + a], (float)r.gp[a]);
    if (pacc) {
        float *acc = pacc + (size_t)k * PACC_STRIDE;
        for (int a = 0; a < 6; a++) atomicAdd(&acc[a], (float)r.Gs[a]);
        atomicAdd(&acc[6], (float)r.glo);
    }
}

// per Gaussian: the summed Gs and glo through the rest of the chain, added to
// the outputs
__global__ __launch_bounds__(BLOCK) void k_project_fin(const float *__restrict__ soa, int64_t K,
                                                       const float *__restrict__ pacc, float *__restrict__ gls,
                                                       float *__restrict__ gq, float *__restrict__ glogit)
{
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= K) return;
    const float *acc = pacc + (size_t)k * PACC_STRIDE;
    const double G6[6] = {acc[0], acc[1], acc[2], acc[3], acc[4], acc[5]};
    const double glo = acc[6];
    if (G6[0] == 0.0 && G6[1] == 0.0 && G6[2] == 0.0 && G6[3] == 0.0 && G6[4] == 0.0 && G6[5] == 0.0 && glo == 0.0)
        return;   // no view passed anything back
    const CovGrad c = cov_grad(gauss_terms(soa, K, k), G6, glo);
    if (gls)
        for (int a = 0; a < 3; a++) gls[3 * k + a] += (float)c.gls[a];
    if (gq)
        for (int a = 0; a < 4; a++) gq[4 * k + a] += (float)c.gq[a];
    if (glogit) glogit[k] += (float)c.glogit;
}

// ============================================================================
// Deterministic backward (rxgs_set_deterministic): every sum below runs in a
// fixed order, so two runs give the same bits.

// out = value (overwrite) or out + value (accumulate)
__device__ __forceinline__ void det_store(float *out, double value, int accum)
{
    *out = accum ? (float)((double)*out + value) : (float)value;
}

// per Gaussian, the views in order (FP64 sums), then the rest of the chain
__global__ __launch_bounds__(BLOCK) void k_det_project(
    const float *__restrict__ soa, int64_t K, int64_t Kp, const float *__restrict__ centres, int V, DevGrid g,
    const int *__restrict__ oinv, const float *__restrict__ g2d, float *__restrict__ gmeans,
    float *__restrict__ gls, float *__restrict__ gq, float *__restrict__ glogit, int accum)
{
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= K) return;
    const GaussTerms t = gauss_terms(soa, K, k);
    const double px = soa[k], py = soa[K + k], pz = soa[2 * K + k];
    double gp[3] = {0.0, 0.0, 0.0}, G6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, glo = 0.0;
    for (int v = 0; v < V; v++) {
        const int s = oinv[(size_t)v * K + k];
        if (s < 0) continue;
        const float *gg = g2d + ((size_t)v * Kp + s) * 8;
        if (g2d_zero(gg)) continue;
        const ViewGrad r = view_grad(px, py, pz, t.S, centres, v, g, gg);
        for (int a = 0; a < 3; a++) gp[a] += r.gp[a];
        for (int a = 0; a < 6; a++) G6[a] += r.Gs[a];
        glo += r.glo;
    }
    const CovGrad c = cov_grad(t, G6, glo);
    if (gmeans)
        for (int a = 0; a < 3; a++) det_store(&gmeans[3 * k + a], gp[a], accum);
    if (gls)
        for (int a = 0; a < 3; a++) det_store(&gls[3 * k + a], c.gls[a], accum);
    if (gq)
        for (int a = 0; a < 4; a++) det_store(&gq[4 * k + a], c.gq[a], accum);
    if (glogit) det_store(&glogit[k], c.glogit, accum);
}

// sorted position of every (view, Gaussian), -1 where not visible
__global__ __launch_bounds__(BLOCK) void k_order_inv(const uint32_t *__restrict__ order,
                                                     const unsigned long long *__restrict__ counters, int V,
                                                     int64_t K, int64_t Kp, int *__restrict__ oinv)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= (int64_t)V * Kp) return;
    const int64_t v = i / Kp, s = i - v * Kp;
    if (s >= (int64_t)counters[2 * (size_t)v]) return;
    const int64_t k = order[i];
    if (k < K) oinv[(size_t)v * K + k] = (int)s;
}

// per (view, visible position): the record gradients summed over the
// position's pairs in emission order (and, within a pair, the receiver blocks
// in order)
__global__ __launch_bounds__(BLOCK) void k_det_gather(const float *__restrict__ gP, int64_t Dpad, int Rdet,
                                                      const uint32_t *__restrict__ poff,
                                                      const uint32_t *__restrict__ pbase,
                                                      const uint32_t *__restrict__ pcount,
                                                      const unsigned long long *__restrict__ counters,
                                                      const int4 *__restrict__ vinfo, int V, int64_t Kp,
                                                      float *__restrict__ g2d)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= (int64_t)V * Kp) return;
    const int v = (int)(i / Kp);
    const int64_t s = i - (int64_t)v * Kp;
    const int64_t nvis = (int64_t)counters[2 * (size_t)v];
    if (s >= nvis) return;
    const uint32_t e0 = poff[i], e1 = s + 1 < nvis ? poff[i + 1] : pcount[v];
    const size_t b0 = pbase[v];
    const int nblk = (vinfo[v].y + Rdet - 1) / Rdet;
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (uint32_t e = e0; e < e1; e++) {
        for (int b = 0; b < nblk; b++) {
            const float4 *src = reinterpret_cast<const float4 *>(gP + ((size_t)b * Dpad + b0 + e) * 8);
            const float4 x = src[0], y = src[1];
            acc[0] += x.x;
            acc[1] += x.y;
            acc[2] += x.z;
            acc[3] += x.w;
            acc[4] += y.x;
            acc[5] += y.y;
        }
    }
    float4 *dst = reinterpret_cast<float4 *>(g2d + (size_t)i * 8);
    dst[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    dst[1] = make_float4(acc[4], acc[5], 0.f, 0.f);
}

// per (row, sorted position of the row's view): dL/ds summed over the
// position's pairs in emission order; marks the position blocks with a
// nonzero dL/ds for the MLP backward
__global__ __launch_bounds__(BLOCK) void k_det_gather_ds(const float *__restrict__ dSP, int64_t Dpad,
                                                         const uint32_t *__restrict__ poff,
                                                         const uint32_t *__restrict__ pbase,
                                                         const uint32_t *__restrict__ pcount,
                                                         const unsigned long long *__restrict__ counters,
                                                         const int4 *__restrict__ vinfo,
                                                         const int *__restrict__ rxview, int64_t Kp,
                                                         float *__restrict__ dS, uint8_t *__restrict__ live)
{
    const int j = blockIdx.y;
    const int v = rxview[j];
    const int64_t nvis = (int64_t)counters[2 * (size_t)v];
    const int rl = j - vinfo[v].x;
    const size_t b0 = pbase[v];
    for (int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x; s < nvis; s += (int64_t)gridDim.x * BLOCK) {
        const size_t i = (size_t)v * Kp + s;
        const uint32_t e0 = poff[i], e1 = s + 1 < nvis ? poff[i + 1] : pcount[v];
        float sx = 0.f, sy = 0.f;
        for (uint32_t e = e0; e < e1; e++) {
            const float2 d = *reinterpret_cast<const float2 *>(dSP + ((size_t)rl * Dpad + b0 + e) * 2);
            sx += d.x;
            sy += d.y;
        }
        *reinterpret_cast<float2 *>(dS + ((size_t)j * Kp + s) * 2) = make_float2(sx, sy);
        if (sx != 0.f || sy != 0.f) live[i / MLP_PAIRS] = 1;
    }
}

// direct radiance: dL/d radiance_k over the rows in order
__global__ __launch_bounds__(BLOCK) void k_det_rad(const float2 *__restrict__ dS, const int *__restrict__ oinv,
                                                   const int *__restrict__ rxview, int N, int64_t K, int64_t Kp,
                                                   float *__restrict__ grad, int accum)
{
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= K) return;
    double ax = 0.0, ay = 0.0;
    for (int j = 0; j < N; j++) {
        const int s = oinv[(size_t)rxview[j] * K + k];
        if (s < 0) continue;
        const float2 d = dS[(size_t)j * Kp + s];
        ax += d.x;
        ay += d.y;
    }
    det_store(&grad[2 * k], ax, accum);
    det_store(&grad[2 * k + 1], ay, accum);
}

// ranks of the marked position blocks in index order (-1 unmarked): counts
// per chunk of 1024 blocks, their exclusive scan (one workgroup), the ranks
__global__ __launch_bounds__(BLOCK) void k_live_count(const uint8_t *__restrict__ live, int64_t nb,
                                                      uint32_t *__restrict__ cnt)
{
    __shared__ uint32_t s_c[BLOCK / 64];
    uint32_t c = 0;
    for (int q = 0; q < 4; q++) {
        const int64_t b = (int64_t)blockIdx.x * 1024 + q * BLOCK + threadIdx.x;
        c += (b < nb && live[b]) ? 1u : 0u;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o);
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
}

__global__ __launch_bounds__(BLOCK) void k_scan_counts(uint32_t *__restrict__ cnt, int64_t n,
                                                       uint32_t *__restrict__ total)
{
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (int64_t i = 0; i < n; i++) {
        const uint32_t c = cnt[i];
        cnt[i] = run;
        run += c;
    }
    *total = run;
}

__global__ __launch_bounds__(BLOCK) void k_live_rank(const uint8_t *__restrict__ live, int64_t nb,
                                                     const uint32_t *__restrict__ off, int *__restrict__ rank)
{
    __shared__ uint32_t s_w[BLOCK / 64];
    uint32_t base = off[blockIdx.x];
    for (int q = 0; q < 4; q++) {
        const int64_t b = (int64_t)blockIdx.x * 1024 + q * BLOCK + threadIdx.x;
        const bool lv = b < nb && live[b];
        const uint64_t m = __ballot(lv);
        if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < (int)(threadIdx.x >> 6); w++) before += s_w[w];
        if (b < nb) rank[b] = lv ? (int)(base + before + (uint32_t)count_below(m)) : -1;
        base += s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
}

// the MLP backward's Gaussian term, per Gaussian and hidden unit: the views
// in order, in each the receiver groups in order
__global__ __launch_bounds__(BLOCK) void k_det_dl(const float *__restrict__ dLv, int nrg_max,
                                                  const int *__restrict__ oinv, const int *__restrict__ rank,
                                                  const int4 *__restrict__ vinfo, int V, int64_t K, int64_t Kp,
                                                  float *__restrict__ dL)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= K * HID) return;
    const int64_t k = i / HID;
    const int u = (int)(i - k * HID);
    float acc = 0.f;
    for (int v = 0; v < V; v++) {
        const int s = oinv[(size_t)v * K + k];
        if (s < 0) continue;
        const int rk = rank[((size_t)v * Kp + s) / MLP_PAIRS];
        if (rk < 0) continue;
        const int nrg = (vinfo[v].y + MLP_RG - 1) / MLP_RG;
        for (int a = 0; a < nrg; a++)
            acc += dLv[(((size_t)rk * nrg_max + a) * MLP_PAIRS + (s % MLP_PAIRS)) * HID + u];
    }
    dL[i] = acc;
}

// ... and its receiver term, per row (one wave, lane = hidden unit): the
// row's marked position blocks in increasing order (64 ranks read at a time,
// the live ones walked through the ballot mask from its lowest bit)
__global__ __launch_bounds__(BLOCK) void k_det_dg(const float *__restrict__ dGp, int rows_max,
                                                  const int *__restrict__ rank, const int *__restrict__ rxview,
                                                  const int4 *__restrict__ vinfo,
                                                  const unsigned long long *__restrict__ counters, int N, int64_t Kp,
                                                  float *__restrict__ dG)
{
    static_assert(HID == 64, "one lane per hidden unit");
    const int j = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= N) return;   // uniform across the wave
    const int v = rxview[j];
    const int rl = j - vinfo[v].x;
    const int64_t nb = ((int64_t)counters[2 * (size_t)v] + MLP_PAIRS - 1) / MLP_PAIRS;
    const int64_t b0 = (int64_t)v * Kp / MLP_PAIRS;
    float acc = 0.f;
    for (int64_t c = 0; c < nb; c += 64) {
        const int64_t b = c + lane;
        const int rk = b < nb ? rank[b0 + b] : -1;
        uint64_t m = __ballot(rk >= 0);
        while (m) {
            const int l = (int)__builtin_ctzll(m);
            m &= m - 1;
            const int r = __builtin_amdgcn_readlane(rk, l);
            acc += dGp[((size_t)r * rows_max + rl) * HID + lane];
        }
    }
    dG[(size_t)j * HID + lane] = acc;
}

// ============================================================================
static inline unsigned nblk(size_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

// zeroes up to ZERO_RANGES buffers in one launch (blockIdx.y picks the range)
__global__ __launch_bounds__(BLOCK) void k_zero_ranges(ZeroRanges z)
{
    const int r = blockIdx.y;
    if (r >= z.n) return;
    uint32_t *p = z.p[r];
    const size_t n = z.len[r];
    for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * BLOCK) p[i] = 0u;
}

// zeroes, per segment y (a view, or a receiver and its view), the words of
// the view's visible positions only: [0, visible(view) x wpr) of the
// segment's Kp x wpr words (nothing reads the rest)
__global__ __launch_bounds__(BLOCK) void k_zero_visible(uint32_t *__restrict__ p, int64_t Kp, int wpr,
                                                        const unsigned long long *__restrict__ counters,
                                                        const int *__restrict__ segview, int nseg)
{
    const int y = blockIdx.y;
    if (y >= nseg) return;
    const int v = segview ? segview[y] : y;
    const size_t n = (size_t)min((int64_t)counters[2 * (size_t)v], Kp) * (size_t)wpr;
    uint32_t *base = p + (size_t)y * (size_t)Kp * (size_t)wpr;
    for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * BLOCK) base[i] = 0u;
}

hipError_t launch_zero_visible(uint32_t *p, int64_t Kp, int wpr, const unsigned long long *counters,
                               const int *segview, int nseg, hipStream_t st)
{
    if (nseg <= 0 || Kp <= 0) return hipSuccess;
    if (nseg > 65535) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)std::min<size_t>(nblk((size_t)Kp * (size_t)wpr), 1024);
    hipLaunchKernelGGL(k_zero_visible, dim3(blocks, (unsigned)nseg), dim3(BLOCK), 0, st, p, Kp, wpr, counters,
                       segview, nseg);
    return hipGetLastError();
}

hipError_t launch_zero_ranges(const ZeroRanges &z, hipStream_t st)
{
    if (z.n <= 0) return hipSuccess;
    if (z.n > ZERO_RANGES) return hipErrorInvalidValue;
    size_t most = 0;
    for (int r = 0; r < z.n; r++) most = std::max(most, z.len[r]);
    if (most == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>(nblk(most), 4096);
    hipLaunchKernelGGL(k_zero_ranges, dim3(blocks, (unsigned)z.n), dim3(BLOCK), 0, st, z);
    return hipGetLastError();
}

template <int R, bool DET>
static hipError_t blend_bwd_launch(Workspace &ws, const float *C, const float *dC, const float *dP, const float *dA,
                                   hipStream_t st)
{
    // forward chunks hold at most ws.R receivers; split them into R-receiver blocks
    const int split = (ws.R + R - 1) / R;
    const int64_t ny = (int64_t)ws.n_chunks * split;
    if (ny > 65535 || ws.g.tiles > 0x7fffffff) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)ws.g.tiles, (unsigned)ny);
    const DetPartials det = DET ? DetPartials{ws.gP.as<float>(), ws.dSP.as<float>(), ws.Dpad, ws.d_vinfo,
                                              ws.sbox.as<float4>(), ws.poff.as<uint32_t>(), ws.d_pbase}
                                : DetPartials{nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr};
    hipLaunchKernelGGL((k_blend_bwd<R, DET>), grid, dim3(BLOCK), 0, st, ws.srec.as<float4>(),
                       ws.pval[ws.pairs_buf].as<uint32_t>(), ws.ranges.as<uint2>(), ws.rad.as<float2>(),
                       ws.d_chunks, split, ws.Kp, ws.g, ws.mode == RXGS_MODE_TX ? 1 : 0, C, dC, dP, dA,
                       ws.Tfin.as<float>(), ws.nlast.as<int>(), ws.dS.as<float>(), ws.g2d.as<float>(),
                       ws.live.as<uint8_t>(), det);
    return hipGetLastError();
}

hipError_t launch_blend_bwd(Workspace &ws, const float *C, const float *dC, const float *dP, const float *dA,
                            hipStream_t st)
{
    if (ws.n_chunks == 0) return hipSuccess;
    if (ws.det) {
        switch (det_block_rows(ws)) {
        case 1: return blend_bwd_launch<1, true>(ws, C, dC, dP, dA, st);
        case 2: return blend_bwd_launch<2, true>(ws, C, dC, dP, dA, st);
        default: return blend_bwd_launch<4, true>(ws, C, dC, dP, dA, st);
        }
    }
    switch (ws.R) {
    case 1: return blend_bwd_launch<1, false>(ws, C, dC, dP, dA, st);
    case 2: return blend_bwd_launch<2, false>(ws, C, dC, dP, dA, st);
    case 4: return blend_bwd_launch<4, false>(ws, C, dC, dP, dA, st);
    default: return blend_bwd_launch<8, false>(ws, C, dC, dP, dA, st);   // 8 and 16
    }
}

// receivers per block of the deterministic blend backward (its per-wave LDS
// slots hold 6 + 2 R values per entry)
int det_block_rows(const Workspace &ws) { return std::min(ws.R, 4); }

// the deterministic backward's gathers of the pair partials per (view,
// position) and per (row, position), and the inverse of the sorted order
hipError_t launch_det_gather(Workspace &ws, hipStream_t st)
{
    const size_t VK = (size_t)ws.V * ws.Kp;
    const unsigned long long *cnt = ws.counters.as<unsigned long long>();
    hipLaunchKernelGGL(k_det_gather, dim3(nblk(VK)), dim3(BLOCK), 0, st, ws.gP.as<float>(), ws.Dpad,
                       det_block_rows(ws), ws.poff.as<uint32_t>(), ws.d_pbase, ws.d_pcount, cnt, ws.d_vinfo, ws.V,
                       ws.Kp, ws.g2d.as<float>());
    if (ws.N > 65535) return hipErrorInvalidConfiguration;
    const unsigned bx = (unsigned)std::min<size_t>(nblk((size_t)ws.Kp), 64);
    hipLaunchKernelGGL(k_det_gather_ds, dim3(bx, (unsigned)ws.N), dim3(BLOCK), 0, st, ws.dSP.as<float>(), ws.Dpad,
                       ws.poff.as<uint32_t>(), ws.d_pbase, ws.d_pcount, cnt, ws.d_vinfo, ws.d_rxview, ws.Kp,
                       ws.dS.as<float>(), ws.live.as<uint8_t>());
    hipLaunchKernelGGL(k_order_inv, dim3(nblk(VK)), dim3(BLOCK), 0, st, ws.vorder.as<uint32_t>(), cnt, ws.V, ws.K,
                       ws.Kp, ws.oinv.as<int>());
    return hipGetLastError();
}

hipError_t launch_live_rank(Workspace &ws, hipStream_t st)
{
    const int64_t nb = (int64_t)ws.V * ws.Kp / MLP_PAIRS;
    const int64_t nch = (nb + 1023) / 1024;
    uint32_t *cnt = ws.lcnt.as<uint32_t>();
    if (nch > 0) {
        hipLaunchKernelGGL(k_live_count, dim3((unsigned)nch), dim3(BLOCK), 0, st, ws.live.as<uint8_t>(), nb, cnt);
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(BLOCK), 0, st, cnt, nch, cnt + nch);
        hipLaunchKernelGGL(k_live_rank, dim3((unsigned)nch), dim3(BLOCK), 0, st, ws.live.as<uint8_t>(), nb, cnt,
                           ws.rank.as<int>());
    }
    return hipGetLastError();
}

size_t live_rank_words(const Workspace &ws) { return (size_t)(((int64_t)ws.V * ws.Kp / MLP_PAIRS + 1023) / 1024) + 1; }

hipError_t launch_det_rad(const Scene &sc, Workspace &ws, float *grad, int accum, hipStream_t st)
{
    if (!grad || sc.K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_det_rad, dim3(nblk((size_t)sc.K)), dim3(BLOCK), 0, st, ws.dS.as<float2>(), ws.oinv.as<int>(),
                       ws.d_rxview, ws.N, sc.K, ws.Kp, grad, accum);
    return hipGetLastError();
}

hipError_t launch_det_mlp_gather(Workspace &ws, hipStream_t st)
{
    const int nrg_max = (std::min(ws.R_max, 1 << 30) + MLP_RG - 1) / MLP_RG;
    if (ws.K > 0)
        hipLaunchKernelGGL(k_det_dl, dim3(nblk((size_t)ws.K * HID)), dim3(BLOCK), 0, st, ws.dLv.as<float>(), nrg_max,
                           ws.oinv.as<int>(), ws.rank.as<int>(), ws.d_vinfo, ws.V, ws.K, ws.Kp, ws.dL.as<float>());
    hipLaunchKernelGGL(k_det_dg, dim3(nblk((size_t)ws.N * HID)), dim3(BLOCK), 0, st, ws.dGp.as<float>(), ws.R_max,
                       ws.rank.as<int>(), ws.d_rxview, ws.d_vinfo, ws.counters.as<unsigned long long>(), ws.N, ws.Kp,
                       ws.dG.as<float>());
    return hipGetLastError();
}

hipError_t launch_det_project(const Scene &sc, Workspace &ws, const rxgs_grads &gr, hipStream_t st)
{
    if (sc.K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_det_project, dim3(nblk((size_t)sc.K)), dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K, ws.Kp,
                       ws.centres_p, ws.V, ws.g, ws.oinv.as<int>(), ws.g2d.as<float>(), gr.means, gr.log_scales,
                       gr.quats, gr.logits, gr.accumulate);
    return hipGetLastError();
}

hipError_t launch_rad_bwd(const Scene &sc, Workspace &ws, float *grad, hipStream_t st)
{
    const int64_t n = (int64_t)ws.N * ws.Kp;
    if (n == 0 || !grad || sc.K == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rad_direct_bwd, dim3(nblk(n)), dim3(BLOCK), 0, st, ws.dS.as<float2>(),
                       ws.vorder.as<uint32_t>(), ws.counters.as<unsigned long long>(),
                       ws.d_rxview, ws.N, ws.Kp, sc.K, grad);
    return hipGetLastError();
}

int mlp_bwd_waves(const Workspace &ws)
{
    const int want = (ws.n_items + 3) / 4;
    return 4 * std::max(1, std::min(want, 256));   // one wave per SIMD fits (372 registers a lane)
}

hipError_t launch_mlp_bwd(const Scene &sc, const Mlp &m, Workspace &ws, float *gfeat, float *gmlp, hipStream_t st)
{
    const float *raw = m.raw.as<float>();
    const float *W1 = raw;
    const float *W3 = raw + HID * MLP_IN + HID + HID * HID + HID;
    const int nwaves = mlp_bwd_waves(ws);
    const bool far = ws.mpos != 0xFFFFFFFFu;   // the forward evaluated a radiance prefix first
    if (far && (int64_t)ws.n_items + ws.n_items_far >= (1ll << 31)) return hipErrorInvalidValue;
    // virtual items per work item: enough that each holds at most MLPB_RSUB receivers
    // (the deterministic backward keeps whole items: one slot per receiver group)
    const int nsub = ws.det ? 1 : (std::min(ws.R_max, MLP_RG) + MLPB_RSUB - 1) / MLPB_RSUB;
    const int64_t nall = (int64_t)ws.n_items + (far ? ws.n_items_far : 0);
    if (nall > INT32_MAX / std::max(nsub, 1)) return hipErrorInvalidValue;   // virtual item indices are int
    // the list of live virtual items (in the reduction scratch, first written
    // after the MLP backward) when every item holds one receiver (views of
    // one receiver: their live items are few and sit at the start of each
    // view's items) and there are at most 256 chunks of 1024; items of several
    // receivers are split into virtual items, which the scattered order
    // already spreads well (the list's two launches would cost more)
    const int64_t nvirt_max = nall * std::max(nsub, 1);
    const int64_t nchunk = (nvirt_max + 4 * BLOCK - 1) / (4 * BLOCK);
    constexpr size_t LIST_AT = 512;   // u32 words: chunk counts, the list length, then the list
    const bool ranked = ws.R_max == 1 && nchunk > 0 && nchunk <= BLOCK &&
                        ws.mred.cap >= (LIST_AT + (size_t)nvirt_max) * 4;
    uint32_t *lw = ranked ? ws.mred.as<uint32_t>() : nullptr;
    const int4 *items2 = far ? ws.items_far.as<int4>() : nullptr;
    const int *count2 = far ? far_count(ws) : nullptr;
    if (ranked) {
        hipLaunchKernelGGL(k_live_list<false>, dim3((unsigned)nchunk), dim3(BLOCK), 0, st, ws.items.as<int4>(),
                           ws.n_items, items2, count2, std::max(nsub, 1), ws.Kp, ws.live.as<uint8_t>(), lw,
                           lw + BLOCK, lw + LIST_AT);
        hipLaunchKernelGGL(k_live_list<true>, dim3((unsigned)nchunk), dim3(BLOCK), 0, st, ws.items.as<int4>(),
                           ws.n_items, items2, count2, std::max(nsub, 1), ws.Kp, ws.live.as<uint8_t>(), lw,
                           lw + BLOCK, lw + LIST_AT);
    }
    if (nall > 0 && ws.det) {
        const DetMlp det{ws.dLv.as<float>(), ws.dGp.as<float>(), ws.rank.as<int>(), ws.d_vinfo,
                         (ws.R_max + MLP_RG - 1) / MLP_RG, ws.R_max};
        hipLaunchKernelGGL(k_mlp_bwd<true>, dim3((unsigned)(nwaves / 4)), dim3(BLOCK), 0, st, ws.Lp.as<float>(),
                           ws.Gp.as<float>(), m.w2a.as<float>(), m.w2b.as<float>(), m.tab.as<float4>(), W3,
                           ws.vorder.as<uint32_t>(), ws.items.as<int4>(), ws.n_items, items2, count2,
                           std::max(nsub, 1), ws.Kp, sc.K, ws.live.as<uint8_t>(), ranked ? lw + LIST_AT : nullptr,
                           ranked ? lw + BLOCK : nullptr, ws.dS.as<float2>(), ws.dL.as<float>(),
                           ws.dG.as<float>(), ws.mpart.as<float>(), det);
        const hipError_t e = launch_det_mlp_gather(ws, st);
        if (e != hipSuccess) return e;
    } else if (nall > 0) {
        hipLaunchKernelGGL(k_mlp_bwd<false>, dim3((unsigned)(nwaves / 4)), dim3(BLOCK), 0, st, ws.Lp.as<float>(),
                           ws.Gp.as<float>(), m.w2a.as<float>(), m.w2b.as<float>(), m.tab.as<float4>(), W3,
                           ws.vorder.as<uint32_t>(), ws.items.as<int4>(), ws.n_items, items2, count2,
                           std::max(nsub, 1), ws.Kp, sc.K, ws.live.as<uint8_t>(), ranked ? lw + LIST_AT : nullptr,
                           ranked ? lw + BLOCK : nullptr, ws.dS.as<float2>(), ws.dL.as<float>(),
                           ws.dG.as<float>(), ws.mpart.as<float>(), DetMlp{});
    }
    if (gmlp) {
        if (nall > 0) {
            hipLaunchKernelGGL(k_colsum_groups, dim3(nblk(4096 + 194), RED_GROUPS), dim3(BLOCK), 0, st,
                               ws.mpart.as<float>(), nwaves, MLPB_PART, 4096 + 194, ws.mred.as<double>());
            hipLaunchKernelGGL(k_mlp_bwd_reduce, dim3(nblk(4096 + 194)), dim3(BLOCK), 0, st, ws.mred.as<double>(),
                               gmlp);
        } else {
            hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(gmlp), 0u, RXGS_MLP_NPARAM, st);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_mlp_w1a, dim3(nblk(HID * (ENC + 1))), dim3(BLOCK), 0, st, ws.dG.as<float>(),
                           ws.rxpos_p, ws.N, gmlp);
        const int nchunks = (int)((sc.K + W1B_CHUNK - 1) / W1B_CHUNK);
        if (nchunks > 0) {
            hipLaunchKernelGGL(k_mlp_w1b_part, dim3((unsigned)nchunks), dim3(BLOCK), 0, st, ws.dL.as<float>(),
                               sc.feat.as<float>(), sc.K, ws.w1part.as<float>());
            hipLaunchKernelGGL(k_colsum_groups, dim3(nblk(HID * FEAT), RED_GROUPS), dim3(BLOCK), 0, st,
                               ws.w1part.as<float>(), nchunks, HID * FEAT, HID * FEAT, ws.mred.as<double>());
            hipLaunchKernelGGL(k_mlp_w1b_reduce, dim3(nblk(HID * FEAT)), dim3(BLOCK), 0, st, ws.mred.as<double>(),
                               gmlp);
        } else {
            hipError_t e = hipSuccess;
            for (int d = 0; d < HID && e == hipSuccess; d++)
                e = launch_fill_u32(reinterpret_cast<uint32_t *>(gmlp + d * MLP_IN + ENC), 0u, FEAT, st);
            if (e != hipSuccess) return e;
        }
    }
    if (gfeat && sc.K > 0)
        hipLaunchKernelGGL(k_mlp_dfeat, dim3((unsigned)((sc.K + DF_CHUNK - 1) / DF_CHUNK)), dim3(BLOCK), 0, st,
                           ws.dL.as<float>(), W1, sc.K, gfeat);
    return hipGetLastError();
}

hipError_t launch_project_bwd(const Scene &sc, Workspace &ws, const rxgs_grads &gr, hipStream_t st)
{
    const int64_t n = (int64_t)ws.V * ws.Kp;
    if (sc.K == 0) return hipSuccess;
    // the covariance and opacity part of the chain is wanted (pacc cleared beforehand)
    const bool cov = gr.log_scales || gr.quats || gr.logits;
    hipLaunchKernelGGL(k_proj_terms, dim3(nblk(sc.K)), dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K,
                       ws.pterm.as<ProjTerm>());
    hipLaunchKernelGGL(k_project_bwd, dim3(nblk(n)), dim3(BLOCK), 0, st, ws.pterm.as<ProjTerm>(), sc.K, ws.Kp,
                       ws.centres_p, ws.V, ws.g, ws.vorder.as<uint32_t>(), ws.counters.as<unsigned long long>(),
                       ws.g2d.as<float>(), gr.means, cov ? ws.pacc.as<float>() : nullptr);
    if (cov)
        hipLaunchKernelGGL(k_project_fin, dim3(nblk(sc.K)), dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K,
                           ws.pacc.as<float>(), gr.log_scales, gr.quats, gr.logits);
    return hipGetLastError();
}

size_t mlp_part_bytes(const Workspace &ws) { return (size_t)mlp_bwd_waves(ws) * MLPB_PART * 4; }
size_t mlp_red_bytes() { return (size_t)RED_GROUPS * MLPB_PART * 8; }
size_t w1b_part_bytes(int64_t K) { return (size_t)std::max<int64_t>((K + W1B_CHUNK - 1) / W1B_CHUNK, 1) * HID * FEAT * 4; }

}  // namespace rxgs
