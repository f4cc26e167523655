// Forward kernels of librxgs for gfx950 (CDNA4, wave64).
//
// Pipeline of one render (Alg. 1 of RxGS, arXiv 2605.24290, with the view
// index added to the sort key):
//   k_gauss_prep   stage 1: view-independent projection terms of every
//                  Gaussian (covariance, opacity, cut-off).
//   k_keys         stage 1: per (view, Gaussian) FP32 depth key with the
//                  near, opacity and conservative elevation culls, and the
//                  depth sort's digit totals.                       [HBM]
//   radix sort     stage 1: per-view stable sort of the depth keys (one
//                  segment per view), 4 passes of 8 bits (sort.hip). [HBM]
//   k_emit1        stage 1: exact FP64 projection of the kept entries in
//                  depth order; visible ones compacted into blend
//                  records, boxes and pair offsets; per chunk its pairs
//                  per tile.                                        [ALU]
//   k_bin_scan,    grids of at most 255 tiles: each chunk's start in every
//   k_bin_pairs    tile list, then each (tile, sorted position) pair placed
//                  directly in its tile list, in depth order.       [ALU]
//   k_emit2 and    larger grids: the pairs emitted in depth order into the
//   radix sort     view's segment, then stably sorted by tile.      [HBM]
//   k_ranges_items [start, end) of each tile's list (and the MLP work items).
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
// Stage 1: projection of one Gaussian onto the angular grid of one view
// (Sec. 4.1 and App. B: azimuth/elevation of the mean, Jacobian-projected
// covariance plus the 0.3 px^2 dilation).  Geometry is evaluated in FP64 from
// the FP32 inputs with fused multiply-adds off, so the key kernel and the
// emission kernel, which both evaluate it, agree bit for bit on every tile
// count (the per-view pair counts of the first size the pair segments of the
// second).

// view-independent part: Sigma = R diag(s^2) R^T, opacity, the largest
// Mahalanobis distance q with o exp(-q/2) >= 1/255, and log2 of the opacity
struct GaussGeo {
    float px, py, pz, o32;
    double S00, S01, S02, S11, S12, S22, qmax, lo2;
};

__device__ __forceinline__ void gauss_geo(const float *__restrict__ soa, int64_t K, int64_t k, GaussGeo &G)
{
#pragma clang fp contract(off)
    G.px = soa[k];
    G.py = soa[K + k];
    G.pz = soa[2 * K + k];
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
    G.S00 = R00 * R00 * s0 + R01 * R01 * s1 + R02 * R02 * s2;
    G.S01 = R00 * R10 * s0 + R01 * R11 * s1 + R02 * R12 * s2;
    G.S02 = R00 * R20 * s0 + R01 * R21 * s1 + R02 * R22 * s2;
    G.S11 = R10 * R10 * s0 + R11 * R11 * s1 + R12 * R12 * s2;
    G.S12 = R10 * R20 * s0 + R11 * R21 * s1 + R12 * R22 * s2;
    G.S22 = R20 * R20 * s0 + R21 * R21 * s1 + R22 * R22 * s2;
    G.o32 = (float)(1.0 / (1.0 + exp(-(double)soa[10 * K + k])));
    G.qmax = 0.0;
    G.lo2 = 0.0;
    if (G.o32 >= ALPHA_MIN) {
        G.qmax = 2.0 * log((double)G.o32 / (double)ALPHA_MIN);
        G.lo2 = log2((double)G.o32);
    }
}

// the view-independent part of every Gaussian, computed once per render (in
// FP64) and read back by the key and emission kernels, 48 bytes per Gaussian:
// position and opacity, then the 3-D covariance, the squared-distance bound
// of the support and log2 opacity rounded to FP32.  The emission gathers these
// terms in depth order; the FP32 rounding (a relative 6e-8) moves the
// projected conic and the binning extents by about 1e-7 relative, far below
// their FP32 storage in the blend record, and the backward differentiates
// the FP64 terms it recomputes from the parameters.
struct alignas(16) GaussGeoPacked {
    float px, py, pz, o32;
    float S00, S01, S02, S11;
    float S12, S22, qmax, lo2;
};

// Also the cull bound of each Gaussian, qcull >= q_max trace(Sigma) (rounded
// up): the vertical variance of any projection is at most
// lambda_max(Sigma) / (rho^2 del^2) + 0.3 px^2 <= trace(Sigma) / (rho^2 del^2) + 0.3.
// It also clears the render's counters and the depth sort's scratch (both
// first used by later kernels of the stream).
__global__ __launch_bounds__(BLOCK) void k_gauss_prep(const float *__restrict__ soa, int64_t K,
                                                      GaussGeoPacked *__restrict__ out, float *__restrict__ qcull,
                                                      uint32_t *__restrict__ z0, size_t n0, uint32_t *__restrict__ z1,
                                                      size_t n1)
{
    {
        const size_t stride = (size_t)gridDim.x * BLOCK;
        const size_t i0 = (size_t)blockIdx.x * BLOCK + threadIdx.x;
        for (size_t i = i0; i < n0; i += stride) z0[i] = 0u;
        for (size_t i = i0; i < n1; i += stride) z1[i] = 0u;
    }
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= K) return;
    GaussGeo G;
    gauss_geo(soa, K, k, G);
    GaussGeoPacked o;
    o.px = G.px; o.py = G.py; o.pz = G.pz; o.o32 = G.o32;
    o.S00 = (float)G.S00; o.S01 = (float)G.S01; o.S02 = (float)G.S02;
    o.S11 = (float)G.S11; o.S12 = (float)G.S12; o.S22 = (float)G.S22;
    o.qmax = (float)G.qmax; o.lo2 = (float)G.lo2;
    out[k] = o;
    qcull[k] = (float)(G.qmax * (G.S00 + G.S11 + G.S22) * (1.0 + 1e-6));
}

__device__ __forceinline__ void gauss_geo_load(const GaussGeoPacked *__restrict__ gg, int64_t k, GaussGeo &G)
{
    const float4 *d = reinterpret_cast<const float4 *>(gg + k);
    const float4 f = d[0], a = d[1], b = d[2];
    G.px = f.x; G.py = f.y; G.pz = f.z; G.o32 = f.w;
    G.S00 = a.x; G.S01 = a.y; G.S02 = a.z; G.S11 = a.w; G.S12 = b.x; G.S22 = b.y;
    G.qmax = b.z; G.lo2 = b.w;
}

// view part: FP32 depth key, grid position, projected covariance (A, B; B, C)
// in px^2, padded binning half-extents and the number of covered tiles
struct ViewGeo {
    uint32_t kb;   // FP32 bits of the squared distance to the view centre
    uint32_t nt;   // covered tiles; 0: culled (near, faint, or off the grid)
    double u, vv, A, B, Cc;
    float4 e;      // binning box (u, v, rup, rvp) in FP32
};

__device__ __forceinline__ void view_geo(const GaussGeo &G, float cx, float cy, float cz, const DevGrid &g,
                                         ViewGeo &P)
{
#pragma clang fp contract(off)
    const float dxf = __fsub_rn(G.px, cx), dyf = __fsub_rn(G.py, cy), dzf = __fsub_rn(G.pz, cz);
    const float kf = depth_key(dxf, dyf, dzf);
    P.kb = __float_as_uint(kf);
    P.nt = 0;
    P.e = make_float4(0.f, 0.f, 0.f, 0.f);
    P.u = P.vv = P.A = P.B = P.Cc = 0.0;
    if (kf < NEAR2) return;
    const double dx = (double)G.px - (double)cx, dy = (double)G.py - (double)cy, dz = (double)G.pz - (double)cz;
    double h = sqrt(dx * dx + dy * dy);
    if (!(h >= H_MIN)) h = H_MIN;
    double az = atan2(dy, dx);
    if (az < 0.0) az += 2.0 * M_PI;
    const double el = atan2(dz, h);
    P.u = az * g.idaz - 0.5;
    P.vv = (el - g.el0) * g.idel - 0.5;
    const double hh = h * h, rh2 = hh + dz * dz;
    // 1 / (h^2 daz) and 1 / (rho^2 h del) from one reciprocal
    const double rhh = rh2 * h;
    const double qd = 1.0 / (hh * rhh);
    const double ihh = g.idaz * (rhh * qd);
    const double irh = g.idel * (hh * qd);
    const double mu0 = -dy * ihh, mu1 = dx * ihh;
    const double mv0 = -dx * dz * irh, mv1 = -dy * dz * irh, mv2 = hh * irh;
    const double Smv0 = G.S00 * mv0 + G.S01 * mv1 + G.S02 * mv2;
    const double Smv1 = G.S01 * mv0 + G.S11 * mv1 + G.S12 * mv2;
    const double Smv2 = G.S02 * mv0 + G.S12 * mv1 + G.S22 * mv2;
    P.A = G.S00 * mu0 * mu0 + 2.0 * G.S01 * mu0 * mu1 + G.S11 * mu1 * mu1 + DILATE;
    P.B = mu0 * Smv0 + mu1 * Smv1;
    P.Cc = mv0 * Smv0 + mv1 * Smv1 + mv2 * Smv2 + DILATE;
    const float u32 = (float)P.u, v32 = (float)P.vv;
    P.e = make_float4(u32, v32, 0.f, 0.f);
    if (G.o32 >= ALPHA_MIN) {
        const float rup = (float)(sqrt(G.qmax * P.A) * (1.0 + PAD_REL) + PAD_ABS);
        const float rvp = (float)(sqrt(G.qmax * P.Cc) * (1.0 + PAD_REL) + PAD_ABS);
        P.e.z = rup;
        P.e.w = rvp;
        int ty0, ty1, a0, a1, b0, b1;
        const int nr = tile_rows(v32, rvp, g.H, ty0, ty1);
        const int nc = nr ? tile_cols(u32, rup, g.W, g.tiles_x, a0, a1, b0, b1) : 0;
        P.nt = (uint32_t)(nr * nc);
    }
}

// blend record of a visible (view, Gaussian): integer and fractional parts of
// the pixel position (pixel offsets stay exact to ~1e-7 px in FP32), the
// inverse projected covariance times -log2(e) (1/2, 1, 1/2), log2 opacity
__device__ __forceinline__ void blend_record(const GaussGeo &G, const ViewGeo &P, float4 &r0, float4 &r1)
{
#pragma clang fp contract(off)
    const double idet = 1.0 / (P.A * P.Cc - P.B * P.B);
    const double ca = P.Cc * idet, cb = -P.B * idet, cc = P.A * idet;
    const double uf = floor(P.u), vf = floor(P.vv);
    constexpr double L2E = 1.4426950408889634;
    r0 = make_float4((float)uf, (float)(P.u - uf), (float)vf, (float)(P.vv - vf));
    r1 = make_float4((float)(-0.5 * L2E * ca), (float)(-L2E * cb), (float)(-0.5 * L2E * cc), (float)G.lo2);
}

// Conservative elevation test in FP32: false only if the Gaussian's padded
// binning box lies entirely below row 0 or above row H - 1 of the grid, which
// the exact FP64 projection would also find.  The half-extent bound uses
// qcull and the 0.3 px^2 dilation with q_max <= 2 ln 255 < 11.1, a relative
// margin for the FP32 evaluation, and 0.01 px for the elevation error of
// atan2f (< 1e-4 px on 1-degree rows).
__device__ __forceinline__ bool maybe_on_grid(float dxf, float dyf, float dzf, float key, float qcull,
                                              const DevGrid &g)
{
    const float h = sqrtf(dxf * dxf + dyf * dyf);
    const float el = atan2f(dzf, h);
    const float vv = (el - (float)g.el0) * (float)g.idel - 0.5f;
    const float idel = (float)g.idel;
    const float R = sqrtf(qcull * idel * idel / key + 3.33f) * 1.0002f + 0.02f;
    return !(vv + R < -0.01f || vv - R > (float)(g.H - 1) + 0.01f);
}

// Depth keys of VPW views' tile of PER x BLOCK Gaussians (PER per thread,
// strided so that loads and stores are coalesced; each Gaussian's terms are
// read once for the VPW views), with the culls of k_project, and the tile's
// contribution to the depth sort's digit totals: LDS counts of all four 8-bit
// digits of the kept keys per view, added to the view's totals with one
// atomic per nonzero count (the values, the Gaussian indices, are not
// written: the sort's first pass takes each key's index in its view's
// segment).  Many views: tiles of 2048 (fewer atomics), four views per
// workgroup for large scenes (whose per-Gaussian terms do not stay in L2);
// few views: tiles of 256 (enough workgroups).
template <int PER, int VPW>
__global__ __launch_bounds__(BLOCK) void k_keys(const GaussGeoPacked *__restrict__ gg,
                                                const float *__restrict__ qcull, int64_t K, int64_t Kp,
                                                const float *__restrict__ centres, DevGrid g, int V,
                                                uint32_t *__restrict__ skey, uint32_t *__restrict__ hist)
{
    constexpr int KEY_TILE = PER * BLOCK;
    __shared__ uint32_t h[VPW][4][256];   // [view][digit position][digit]
    const int t = threadIdx.x;
    const int64_t tiles = Kp / KEY_TILE;
    const int vg = (int)(blockIdx.x / (uint64_t)tiles);
    const int64_t k0 = (int64_t)(blockIdx.x - (uint64_t)vg * (uint64_t)tiles) * KEY_TILE;
    const int v0 = vg * VPW;
#pragma unroll
    for (int vv = 0; vv < VPW; vv++)
#pragma unroll
        for (int p = 0; p < 4; p++) h[vv][p][t] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; r++) {
        const int64_t k = k0 + r * BLOCK + t;
        float4 po = make_float4(0.f, 0.f, 0.f, 0.f);
        float qc = 0.f;
        if (k < K) {
            po = *reinterpret_cast<const float4 *>(gg + k);
            qc = qcull[k];
        }
#pragma unroll
        for (int vv = 0; vv < VPW; vv++) {
            const int v = v0 + vv;
            if (v >= V) break;
            uint32_t key = 0xFFFFFFFFu;
            if (k < K) {
                const float cx = centres[3 * v], cy = centres[3 * v + 1], cz = centres[3 * v + 2];
                const float dxf = __fsub_rn(po.x, cx), dyf = __fsub_rn(po.y, cy), dzf = __fsub_rn(po.z, cz);
                const float kf = depth_key(dxf, dyf, dzf);
                if (!(kf < NEAR2) && po.w >= ALPHA_MIN && maybe_on_grid(dxf, dyf, dzf, kf, qc, g))
                    key = __float_as_uint(kf);
            }
            skey[(size_t)v * Kp + k] = key;
            if (key != 0xFFFFFFFFu)
#pragma unroll
                for (int p = 0; p < 4; p++) atomicAdd(&h[vv][p][(key >> (8 * p)) & 255u], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int vv = 0; vv < VPW; vv++) {
        const int v = v0 + vv;
        if (v >= V) break;
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const uint32_t c = h[vv][p][t];
            if (c) atomicAdd(&hist[((size_t)v * 4 + p) * 256 + t], c);
        }
    }
}

// Depth keys of every (view, Gaussian): one thread per Gaussian (coalesced
// loads), looping over a chunk of views.  A key is dropped (0xFFFFFFFF) when
// the Gaussian is too near (FP32 key below 0.2^2 m^2), too faint (opacity
// below 1/255) or surely off the grid's rows; the emission kernel applies the
// exact test to the rest.  SAVE: the exact binning boxes, raw keys and
// opacities are written for export; KEYS = false: only those (a saved
// state's export, computed when first asked for; a render's keys come from
// k_keys, which applies the same culls).
template <bool SAVE, bool KEYS = true>
__global__ __launch_bounds__(BLOCK) void k_project(
    const GaussGeoPacked *__restrict__ gg, const float *__restrict__ qcull, int64_t K, int64_t Kp,
    const float *__restrict__ centres, int V, int vchunk, DevGrid g, uint32_t *__restrict__ skey,
    uint32_t *__restrict__ sval, float4 *__restrict__ ext, uint32_t *__restrict__ rawkey, float *__restrict__ opac,
    uint32_t *__restrict__ z0, size_t n0, uint32_t *__restrict__ z1, size_t n1)
{
    {
        // clears the render's counters and the depth sort's scratch (both
        // first used by later kernels of the stream)
        const size_t stride = (size_t)gridDim.x * gridDim.y * BLOCK;
        const size_t i0 = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * BLOCK + threadIdx.x;
        for (size_t i = i0; i < n0; i += stride) z0[i] = 0u;
        for (size_t i = i0; i < n1; i += stride) z1[i] = 0u;
    }
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int v0 = blockIdx.y * vchunk;
    const int v1 = min(V, v0 + vchunk);
    const bool real = k < K;
    GaussGeo G;
    float4 po = make_float4(0.f, 0.f, 0.f, 0.f);
    float qc = 0.f;
    if (real) {
        if (SAVE) {
            gauss_geo_load(gg, k, G);
            po = make_float4(G.px, G.py, G.pz, G.o32);
        } else {
            po = *reinterpret_cast<const float4 *>(gg + k);
        }
        qc = qcull[k];
    }
    for (int v = v0; v < v1; v++) {
        const size_t i = (size_t)v * Kp + k;
        uint32_t key = 0xFFFFFFFFu, kb = 0xFFFFFFFFu;
        if (real) {
            const float cx = centres[3 * v], cy = centres[3 * v + 1], cz = centres[3 * v + 2];
            const float dxf = __fsub_rn(po.x, cx), dyf = __fsub_rn(po.y, cy), dzf = __fsub_rn(po.z, cz);
            const float kf = depth_key(dxf, dyf, dzf);
            kb = __float_as_uint(kf);
            if (!(kf < NEAR2) && po.w >= ALPHA_MIN && maybe_on_grid(dxf, dyf, dzf, kf, qc, g)) key = kb;
        }
        if (KEYS) {
            skey[i] = key;
            sval[i] = (uint32_t)k;
        }
        if (SAVE) {
            ViewGeo P;
            P.e = make_float4(0.f, 0.f, 0.f, 0.f);
            if (real) view_geo(G, centres[3 * v], centres[3 * v + 1], centres[3 * v + 2], g, P);
            ext[i] = P.e;
            rawkey[i] = kb;
            opac[i] = real ? po.w : 0.f;
        }
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

// Emission, part 1 (after the depth sort): the exact projection of every kept
// entry in depth order.  Workgroups take the views' chunks chunk by chunk
// (workgroup i: chunk i / V of view i mod V, so that the workgroups resident
// together hold the first chunks of many views, and a later chunk's
// look-back mostly finds its predecessors done), each of NT x PER sorted
// entries (PER consecutive ones per thread; 1024 when there
// are many chunks, which amortises each chunk's look-back, 256 for small
// launches, which keeps the chain of chunks short); it loads its entries'
// Gaussian indices before it knows how many the sort kept (the depth sort's
// first pass left that count per view), evaluates them (FP64, the same code as the key kernel's exports)
// and compacts the visible ones (at least one tile covered): their depth rank
// among the view's visible Gaussians and their first pair slot come from one
// workgroup scan of the per-thread (visible, pairs) counts plus a
// wave-parallel decoupled look-back over the view's earlier chunks (one 64-bit
// status word per chunk: flags, visible count, pair count).  Each visible
// entry writes its blend record, binning box, Gaussian index and first pair
// slot at its rank; the view's last chunk writes the view's visible and pair
// counts.  Errors (a look-back that does not end, more than 2^32 - 1 pairs in
// a view) set bits of the error word, which the host checks.
constexpr uint64_t EM_AGG = 1ull << 62, EM_PRE = 1ull << 63;
constexpr int EM_SPIN_MAX = 1 << 20;

__device__ __forceinline__ uint64_t em_pack(uint64_t flag, uint32_t vis, uint32_t pairs)
{
    return flag | ((uint64_t)(vis & 0x3FFFFFFFu) << 32) | pairs;
}

// exclusive scan of two counts at once over a workgroup of NW waves
template <int NW>
__device__ __forceinline__ uint2 block_exclusive_scan2(uint32_t x, uint32_t y, uint2 &total, uint2 *s_w)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t a = x, b = y;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t ya = __shfl_up(a, off), yb = __shfl_up(b, off);
        if (lane >= off) {
            a += ya;
            b += yb;
        }
    }
    if (lane == 63) s_w[w] = make_uint2(a, b);
    __syncthreads();
    uint2 pre = make_uint2(0u, 0u), tot = make_uint2(0u, 0u);
#pragma unroll
    for (int i = 0; i < NW; i++) {
        const uint2 c = s_w[i];
        if (i < w) {
            pre.x += c.x;
            pre.y += c.y;
        }
        tot.x += c.x;
        tot.y += c.y;
    }
    total = tot;
    __syncthreads();
    return make_uint2(pre.x + a - x, pre.y + b - y);
}

// NT threads per workgroup, EM1_PER entries per thread
template <int EM1_PER, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_emit1(
    const GaussGeoPacked *__restrict__ gg, int64_t K, int64_t Kp, const float *__restrict__ centres, DevGrid g,
    const uint32_t *__restrict__ order, const uint32_t *__restrict__ kept, int cpv,
    float4 *__restrict__ srec, float4 *__restrict__ sbox, uint32_t *__restrict__ vorder, uint32_t *__restrict__ poff,
    unsigned long long *__restrict__ counters, unsigned long long *status, uint32_t *err,
    uint32_t limit, uint32_t *__restrict__ vflag, uint32_t *__restrict__ bcnt, uint4 *__restrict__ binfo)
{
    constexpr int NW = NT / 64;
    __shared__ uint2 s_w2[NW];
    __shared__ uint32_t s_vbase, s_pbase;
    __shared__ int s_d[BIN_DIFF_WORDS];
    constexpr int EM1_CHUNK = NT * EM1_PER;
    const int t = threadIdx.x;
    const uint32_t nviews = gridDim.x / (unsigned)cpv;
    const uint32_t chunk = blockIdx.x / nviews;
    const int v = (int)(blockIdx.x - chunk * nviews);
    const int dw = g.tiles_x + 1;   // row stride of the per-tile difference counts
    const int64_t s0 = (int64_t)chunk * EM1_CHUNK;
    const int64_t sb = s0 + (int64_t)t * EM1_PER;
    // the chunk's sorted Gaussian indices, loaded before the kept count is
    // known (positions past it are dropped below; the index is clamped before use)
    uint32_t kk[EM1_PER], nt[EM1_PER];
#pragma unroll
    for (int j = 0; j < EM1_PER; j++) kk[j] = sb + j < Kp ? order[(size_t)v * Kp + sb + j] : 0xFFFFFFFFu;
    // entries the depth sort kept for this view; only the nearest `limit` of
    // them are emitted: record whether that cut any
    const uint32_t kv = kept[(size_t)v * KEPT_STRIDE];
    const uint32_t seg_n = min(kv, limit);
    if (t == 0 && chunk == 0) vflag[v] = kv > limit ? 1u : 0u;
    // uniform; the view's later chunks are past the end too
    if (s0 >= (int64_t)seg_n) return;
    if (bcnt) {
        for (int i = t; i < g.tiles_y * dw; i += NT) s_d[i] = 0;
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < EM1_PER; j++)
        if (sb + j >= (int64_t)seg_n) kk[j] = 0xFFFFFFFFu;
    const float cx = centres[3 * v], cy = centres[3 * v + 1], cz = centres[3 * v + 2];
    float4 r0[EM1_PER], r1[EM1_PER], box[EM1_PER];
    uint32_t nvis = 0, npairs = 0;
#pragma unroll
    for (int j = 0; j < EM1_PER; j++) {
        nt[j] = 0;
        r0[j] = r1[j] = box[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (kk[j] != 0xFFFFFFFFu) {
            kk[j] = (uint32_t)min((int64_t)kk[j], K - 1);
            GaussGeo G;
            gauss_geo_load(gg, kk[j], G);
            ViewGeo P;
            view_geo(G, cx, cy, cz, g, P);
            if (P.nt) {
                nt[j] = P.nt;
                box[j] = P.e;
                blend_record(G, P, r0[j], r1[j]);
                nvis++;
            }
        }
        npairs += nt[j];
    }
    uint2 tot;
    const uint2 pre = block_exclusive_scan2<NW>(nvis, npairs, tot, s_w2);
    if (t < 64) {
        uint32_t evis = 0;
        uint64_t epairs = 0;
        unsigned long long *mine = status + (size_t)v * cpv + chunk;
        if (chunk == 0) {
            if (t == 0) __hip_atomic_store(mine, em_pack(EM_PRE, tot.x, tot.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (t == 0) __hip_atomic_store(mine, em_pack(EM_AGG, tot.x, tot.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // 64 predecessors per step (lane l reads chunk j - l; before the
            // view's first chunk counts as an empty prefix)
            int j = (int)chunk - 1;
            int spins = 0;
            while (true) {
                const int idx = j - t;
                const uint64_t sv = idx >= 0 ? __hip_atomic_load(status + (size_t)v * cpv + idx, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT)
                                             : EM_PRE;
                const uint64_t pre_mask = __ballot((sv & EM_PRE) != 0);
                const int lp = pre_mask ? __builtin_ctzll(pre_mask) : 63;
                const uint64_t upto = lp == 63 ? ~0ull : ((2ull << lp) - 1);
                if (__ballot(sv == 0) & upto) {
                    if (++spins > EM_SPIN_MAX) {
                        if (t == 0) atomicOr(err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                evis += wave_sum_u32(t <= lp ? (uint32_t)((sv >> 32) & 0x3FFFFFFFu) : 0u);
                const uint32_t pv = t <= lp ? (uint32_t)sv : 0u;
                const uint32_t lo = wave_sum_u32(pv & 0xFFFFu), hi = wave_sum_u32(pv >> 16);
                epairs += (uint64_t)lo + ((uint64_t)hi << 16);
                if (pre_mask) break;
                j -= 64;
            }
            if (epairs + tot.y > 0xFFFFFFFFull) {
                if (t == 0) atomicOr(err, 2u);
                epairs = 0;
            }
            if (t == 0)
                __hip_atomic_store(mine, em_pack(EM_PRE, evis + tot.x, (uint32_t)epairs + tot.y), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (t == 0) {
            s_vbase = evis;
            s_pbase = (uint32_t)epairs;
        }
    }
    if (bcnt) {
        // this chunk's pairs per tile (while wave 0 looks back): +1 / -1 at
        // the ends of each covered column run, row by row, then a prefix
        // along each row
#pragma unroll
        for (int j = 0; j < EM1_PER; j++) {
            if (!nt[j]) continue;
            int ty0, ty1, a0, a1, b0, b1;
            (void)tile_rows(box[j].y, box[j].w, g.H, ty0, ty1);
            (void)tile_cols(box[j].x, box[j].z, g.W, g.tiles_x, a0, a1, b0, b1);
            for (int ty = ty0; ty <= ty1; ty++) {
                int *d = s_d + ty * dw;
                atomicAdd(d + a0, 1);
                atomicAdd(d + a1 + 1, -1);
                if (b1 >= b0) {
                    atomicAdd(d + b0, 1);
                    atomicAdd(d + b1 + 1, -1);
                }
            }
        }
    }
    __syncthreads();
    if (bcnt && t < g.tiles) {
        const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
        int c = 0;
        for (int x = 0; x <= tx; x++) c += s_d[ty * dw + x];
        bcnt[((size_t)v * cpv + chunk) * 256 + t] = (uint32_t)c;
    }
    size_t q = (size_t)v * Kp + s_vbase + pre.x;
    uint32_t po = s_pbase + pre.y;
#pragma unroll
    for (int j = 0; j < EM1_PER; j++) {
        if (nt[j]) {
            srec[2 * q] = r0[j];
            srec[2 * q + 1] = r1[j];
            sbox[q] = box[j];
            vorder[q] = kk[j];
            poff[q] = po;
            q++;
            po += nt[j];
        }
    }
    if (t == 0 && s0 + EM1_CHUNK >= (int64_t)seg_n) {
        counters[2 * (size_t)v] = s_vbase + tot.x;
        counters[2 * (size_t)v + 1] = (uint64_t)s_pbase + tot.y;
    }
    if (binfo && t == 0) binfo[(size_t)v * cpv + chunk] = make_uint4(s_vbase, tot.x, s_pbase, tot.y);
}

// Emission, part 2 for grids of more than BIN_MAX_TILES tiles (after the
// counts are known): one (local tile id, sorted position) pair per covered
// tile of every visible entry, in depth order, into the view's segment of the
// pair arrays (segments start at multiples of 4096 so the pair sort can treat
// each view on its own).  One workgroup per
// EM2_CHUNK visible entries of a view, taken 256 at a time; the first pair
// slots come from part 1, and for each window of 2048 output slots an LDS
// table records which entry owns each slot, so consecutive threads write
// consecutive slots.  The chunk holding the view's last entry writes the
// segment's padding keys.
constexpr int EMIT_WIN = 2048;

__global__ __launch_bounds__(BLOCK) void k_emit2(const float4 *__restrict__ sbox, const uint32_t *__restrict__ poff,
                                                 int64_t Kp, DevGrid g,
                                                 const unsigned long long *__restrict__ counters,
                                                 const uint32_t *__restrict__ pbase,
                                                 const uint32_t *__restrict__ pcount,
                                                 const uint32_t *__restrict__ chunk_off, int V,
                                                 uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval,
                                                 uint32_t *__restrict__ zs, size_t nzs)
{
    // clears the pair sort's scratch (first used by the next kernel)
    for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < nzs; i += (size_t)gridDim.x * BLOCK) zs[i] = 0u;
    __shared__ unsigned char s_own[EMIT_WIN];
    __shared__ uint32_t s_pre[BLOCK];
    __shared__ int4 s_tp[BLOCK];     // ty0, a0, columns in range a, b0
    __shared__ float2 s_ncol[BLOCK]; // columns, 1 / columns
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x;
    // the view owning this chunk: the last view whose first chunk is at or
    // before it, i.e. the number of views after the first with that property
    // (chunk_off is non-decreasing), counted in one parallel pass
    uint32_t cnt = 0;
    for (int i = 1 + t; i < V; i += BLOCK) cnt += chunk_off[i] <= blockIdx.x ? 1u : 0u;
    uint32_t vcount;
    (void)block_exclusive_scan(cnt, vcount, s_w);
    const int v = (int)vcount;
    const int64_t c0s = (int64_t)(blockIdx.x - chunk_off[v]) * EM2_CHUNK;
    const int64_t nv = (int64_t)counters[2 * (size_t)v];
    const uint32_t pb = pbase[v], seg_end = pb + pcount[v];
    const size_t row = (size_t)v * Kp;
    float4 e[EM2_PER];
#pragma unroll
    for (int j = 0; j < EM2_PER; j++) {
        const int64_t s = c0s + j * BLOCK + t;
        e[j] = s < nv ? sbox[row + s] : make_float4(0.f, 0.f, -1.f, -1.f);
    }
#pragma unroll
    for (int j = 0; j < EM2_PER; j++) {
        const int64_t s0 = c0s + j * BLOCK;
        if (s0 >= nv) break;   // uniform
        const int64_t s = s0 + t;
        uint32_t nt = 0;
        int4 tp = make_int4(0, 0, 0, 0);
        int ncol = 1;
        if (s < nv) {
            int ty0, ty1, a0, a1, b0, b1;
            const int nr = tile_rows(e[j].y, e[j].w, g.H, ty0, ty1);
            const int nc = nr ? tile_cols(e[j].x, e[j].z, g.W, g.tiles_x, a0, a1, b0, b1) : 0;
            if (nr && nc) {
                nt = (uint32_t)(nr * nc);
                ncol = nc;
                tp = make_int4(ty0, a0, a1 - a0 + 1, b0);
            }
        }
        // (the scan's barriers also order this sub-chunk's table writes after
        // the previous sub-chunk's reads)
        uint32_t tot;
        const uint32_t pre = block_exclusive_scan(nt, tot, s_w);
        s_pre[t] = pre;
        s_tp[t] = tp;
        s_ncol[t] = make_float2((float)ncol, 1.0f / (float)ncol);
        const uint32_t out0 = pb + poff[row + s0];
        const size_t p0 = row + (size_t)s0;
        for (uint32_t c0 = 0; c0 < tot; c0 += EMIT_WIN) {
            __syncthreads();
            const uint32_t a = max(pre, c0), b = min(pre + nt, c0 + (uint32_t)EMIT_WIN);
            for (uint32_t x = a; x < b; x++) s_own[x - c0] = (unsigned char)t;
            __syncthreads();
            const uint32_t cend = min(tot, c0 + (uint32_t)EMIT_WIN);
            for (uint32_t i = c0 + t; i < cend; i += BLOCK) {
                const int r = s_own[i - c0];
                const int4 q = s_tp[r];
                const float2 nc = s_ncol[r];
                const int jj = (int)(i - s_pre[r]);
                // jj / columns through the reciprocal (exact after the
                // correction: jj < 2^24, the quotient is off by at most one)
                int row_i = (int)((float)jj * nc.y);
                int cc = jj - row_i * (int)nc.x;
                if (cc < 0) {
                    row_i--;
                    cc += (int)nc.x;
                } else if (cc >= (int)nc.x) {
                    row_i++;
                    cc -= (int)nc.x;
                }
                const int ty = q.x + row_i;
                const int tx = cc < q.z ? q.y + cc : q.w + (cc - q.z);
                const uint32_t o = out0 + i;
                if (o < seg_end) {
                    pkey[o] = (uint32_t)(ty * g.tiles_x + tx);
                    pval[o] = (uint32_t)(p0 + r);
                }
            }
        }
    }
    if (c0s + EM2_CHUNK >= nv) {
        // this chunk holds the view's last entry: pad the segment to a whole unit
        const uint32_t pend = pb + (uint32_t)(((uint64_t)pcount[v] + SORT_TILE - 1) / SORT_TILE * SORT_TILE);
        for (uint32_t o = seg_end + t; o < pend; o += BLOCK) pkey[o] = 0xFFFFFFFFu;
    }
}

// Direct binning (grids of at most BIN_MAX_TILES tiles): each tile's list is
// written in its final place, in depth order, without a sort of the pairs.
// The first emission counts each chunk's pairs per tile.  Per view,
// k_bin_scan turns those counts into each chunk's start inside every tile's
// list (the counts of the view's earlier chunks) and the view's list
// lengths.  k_bin_pairs then places the pairs in units of BIN_WIN pair slots
// of one chunk (the slots of a chunk are its entries' covered tiles, entry
// by entry in depth order, each entry's tiles row by row): a tile's list
// starts at the view's segment start plus the lengths of the lists of lower
// tiles, a chunk's pairs of that tile follow the earlier chunks', and a
// unit's follow the chunk's slots before the unit.  Inside a unit the pairs
// keep slot order (an entry covers a tile at most once, so this is depth
// order).  The result is the stable sort of the emitted pairs by tile.
//
// One workgroup per view.  Per tile (one thread each): each live chunk's
// count becomes the count of the view's earlier chunks (chunks read
// BIN_SCAN_WIDE, then BIN_SCAN_BATCH at a time, all in flight together) and
// the total is the tile's list length.  Per live chunk: the index of its first group of
// units (up to `group` units, one workgroup of k_bin_pairs) within the view
// (exclusive prefix, nlive + 1 words).
constexpr int BIN_SCAN_BATCH = 16, BIN_SCAN_WIDE = 64;

__global__ __launch_bounds__(BLOCK) void k_bin_scan(const uint32_t *__restrict__ hist, int passes, uint32_t limit,
                                                    int cpv, int chunk, int tiles, int group,
                                                    const uint4 *__restrict__ binfo,
                                                    uint32_t *__restrict__ bcnt, uint32_t *__restrict__ btot,
                                                    uint32_t *__restrict__ blive, uint32_t *__restrict__ bunit)
{
    __shared__ uint32_t s_w[4];
    const int v = blockIdx.x, t = threadIdx.x;
    // live chunks of the view: those holding some of its kept entries
    uint32_t kept;
    (void)block_exclusive_scan(hist[((size_t)v * passes) * 256 + t], kept, s_w);
    const uint32_t nlive = (min(kept, limit) + (uint32_t)chunk - 1) / (uint32_t)chunk;
    if (t == 0) blive[v] = nlive;
    uint32_t *wp = bunit + (size_t)v * (cpv + 1);
    uint32_t ubase = 0;
    for (uint32_t j0 = 0; j0 < nlive; j0 += BLOCK) {   // uniform
        const uint32_t j = j0 + t;
        const uint32_t n = j < nlive ? (binfo[(size_t)v * cpv + j].w + BIN_WIN * group - 1) / (BIN_WIN * group)
                                     : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(n, tot, s_w);
        if (j < nlive) wp[j] = ubase + ex;
        ubase += tot;
    }
    if (t == 0) wp[nlive] = ubase;
    if (t >= tiles) return;
    uint32_t run = 0;
    uint32_t *col = bcnt + (size_t)v * cpv * 256 + t;
    uint32_t j0 = 0;
    // whole batches of BIN_SCAN_WIDE chunks (no per-chunk bound tests), then the rest
    for (; j0 + BIN_SCAN_WIDE <= nlive; j0 += BIN_SCAN_WIDE) {
        uint32_t c[BIN_SCAN_WIDE];
#pragma unroll
        for (int q = 0; q < BIN_SCAN_WIDE; q++) c[q] = col[(size_t)(j0 + q) * 256];
#pragma unroll
        for (int q = 0; q < BIN_SCAN_WIDE; q++) {
            col[(size_t)(j0 + q) * 256] = run;
            run += c[q];
        }
    }
    for (; j0 < nlive; j0 += BIN_SCAN_BATCH) {
        uint32_t c[BIN_SCAN_BATCH];
#pragma unroll
        for (int q = 0; q < BIN_SCAN_BATCH; q++) c[q] = j0 + q < nlive ? col[(size_t)(j0 + q) * 256] : 0u;
#pragma unroll
        for (int q = 0; q < BIN_SCAN_BATCH; q++) {
            if (j0 + q < nlive) col[(size_t)(j0 + q) * 256] = run;
            run += c[q];
        }
    }
    btot[(size_t)v * 256 + t] = run;
}

// +1 / -1 at the ends of the column runs [a0, a1] and [b0, b1] of tile row ty
__device__ __forceinline__ void bin_diff_row(int *s_d, int dw, int ty, int a0, int a1, int b0, int b1)
{
    int *d = s_d + ty * dw;
    atomicAdd(d + a0, 1);
    atomicAdd(d + a1 + 1, -1);
    if (b1 >= b0) {
        atomicAdd(d + b0, 1);
        atomicAdd(d + b1 + 1, -1);
    }
}

// One workgroup per group of up to `group` consecutive units of one chunk
// (heavy chunks, the nearest entries of a view, spread over several; groups
// of one unit when there are few chunks, so heavy chunks spread widely).  The
// chunk's entries' first slots go to LDS; the slots before the group are
// counted per tile (difference counts of whole entries, and of the first rows
// and columns of the entry the group starts in); the group's entries leave
// their tile rectangles in LDS.  Per unit, the entries that start inside it
// are marked in a bitmap of its slots, and each wave takes a contiguous part
// of the unit 64 slots at a time: a slot's entry is the
// number of marks up to it, its tile follows from its rank inside that
// entry's rectangle; the wave ranks its slots by tile (match_key8 and a
// per-wave count per tile in LDS), and the waves' counts give each wave its
// start in every tile's list; the unit's counts advance the starts for the
// next unit.
__global__ __launch_bounds__(BLOCK) void k_bin_pairs(const float4 *__restrict__ sbox,
                                                     const uint32_t *__restrict__ poff, int64_t Kp, DevGrid g,
                                                     int cpv, int V, int group, const uint32_t *__restrict__ uoff,
                                                     const uint4 *__restrict__ binfo,
                                                     const uint32_t *__restrict__ bcnt,
                                                     const uint32_t *__restrict__ btot,
                                                     const uint32_t *__restrict__ blive,
                                                     const uint32_t *__restrict__ bunit,
                                                     const uint32_t *__restrict__ pbase,
                                                     const uint32_t *__restrict__ pcount, uint32_t *__restrict__ pval)
{
    __shared__ uint32_t s_off[BIN_CHUNK_MAX];     // first slot of each entry of the chunk (chunk-relative)
    __shared__ uint32_t s_rect[BIN_CHUNK_MAX];    // per entry of the units: ty0, a0, columns in range a, columns
    __shared__ uint32_t s_mark[BIN_WIN / 32];     // slots of the unit where an entry after the first starts
    __shared__ uint32_t s_mpre[BIN_WIN / 32];     // marks in the words before each word
    __shared__ int s_d[BIN_DIFF_WORDS];           // difference counts of the chunk's slots before the unit
    __shared__ uint32_t s_wc[4][256];             // per wave: its pairs per tile, then its start in each list
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_probe, s_j, s_ea, s_eb, s_ej;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    // the view of this group of units: the number of views after the first whose units
    // start at or before it (uoff is non-decreasing)
    uint32_t cnt = 0;
    for (int i = 1 + t; i < V; i += BLOCK) cnt += uoff[i] <= blockIdx.x ? 1u : 0u;
    uint32_t vcount;
    (void)block_exclusive_scan(cnt, vcount, s_w);
    const int v = (int)vcount;
    const uint32_t u = blockIdx.x - uoff[v];
    const uint32_t nl = blive[v];
    const uint32_t *wp = bunit + (size_t)v * (cpv + 1);
    if (u >= wp[nl]) return;   // uniform: past the view's units
    // its chunk j (wp[j] <= u < wp[j + 1]): every stride-th chunk probed,
    // then the chunks of the bracket
    const uint32_t stride = (nl + BLOCK - 1) / BLOCK;
    if (t == 0) s_probe = 0;
    if (t < BIN_WIN / 32) s_mark[t] = 0;
    __syncthreads();
    {
        const uint32_t c = (uint32_t)t * stride;
        if (c < nl && wp[c] <= u) atomicMax(&s_probe, c);
    }
    __syncthreads();
    for (uint32_t c = s_probe + t; c < min(nl, s_probe + stride); c += BLOCK)
        if (wp[c] <= u && u < wp[c + 1]) s_j = c;
    const int dw = g.tiles_x + 1;
    for (int i = t; i < g.tiles_y * dw; i += BLOCK) s_d[i] = 0;
#pragma unroll
    for (int ww = 0; ww < 4; ww++) s_wc[ww][t] = 0;
    __syncthreads();
    const uint32_t j = s_j;
    const uint4 bi = binfo[(size_t)v * cpv + j];
    const uint32_t nvis = bi.y, pj = bi.w;
    // this workgroup's units of the chunk and their slots
    const uint32_t nu = (pj + BIN_WIN - 1) / BIN_WIN;
    const uint32_t ua = (u - wp[j]) * (uint32_t)group, ub = min(nu, ua + (uint32_t)group);
    const uint32_t sa = ua * BIN_WIN, sz = min(pj, ub * BIN_WIN);
    const size_t row = (size_t)v * Kp + bi.x;
    for (uint32_t e = t; e < nvis; e += BLOCK) s_off[e] = poff[row + e] - bi.z;
    __syncthreads();
    // the entries holding the first and the last of these slots
    for (uint32_t e = t; e < nvis; e += BLOCK) {
        const uint32_t o0 = s_off[e], o1 = e + 1 < nvis ? s_off[e + 1] : pj;
        if (o0 <= sa && sa < o1) s_ea = e;
        if (o0 <= sz - 1 && sz - 1 < o1) s_eb = e;
    }
    __syncthreads();
    const uint32_t ea = s_ea, eb = s_eb;
    // the boxes of entries 0 .. eb (at most four per thread, loaded together)
    constexpr int EPT = BIN_CHUNK_MAX / BLOCK;
    float4 bx[EPT];
#pragma unroll
    for (int q = 0; q < EPT; q++) {
        const uint32_t e = (uint32_t)t + (uint32_t)q * BLOCK;
        bx[q] = e <= eb ? sbox[row + e] : make_float4(0.f, 0.f, -1.f, -1.f);
    }
#pragma unroll
    for (int q = 0; q < EPT; q++) {
        const uint32_t e = (uint32_t)t + (uint32_t)q * BLOCK;
        if (e > eb) continue;
        int ty0, ty1, a0, a1, b0, b1;
        (void)tile_rows(bx[q].y, bx[q].w, g.H, ty0, ty1);
        (void)tile_cols(bx[q].x, bx[q].z, g.W, g.tiles_x, a0, a1, b0, b1);
        const int na = a1 - a0 + 1, nc = na + (b1 - b0 + 1);
        if (e < ea) {   // slots before the first unit: all of this entry's
            for (int ty = ty0; ty <= ty1; ty++) bin_diff_row(s_d, dw, ty, a0, a1, b0, b1);
            continue;
        }
        if (e == ea) {   // its first k slots: whole rows, then the first q columns of the next
            const int k = (int)(sa - s_off[e]);
            const int full = k / nc, qq = k - full * nc;
            for (int ty = ty0; ty < ty0 + full; ty++) bin_diff_row(s_d, dw, ty, a0, a1, b0, b1);
            if (qq > 0) {
                if (qq <= na) bin_diff_row(s_d, dw, ty0 + full, a0, a0 + qq - 1, 0, -1);
                else bin_diff_row(s_d, dw, ty0 + full, a0, a1, b0, b0 + (qq - na) - 1);
            }
        }
        s_rect[e] = (uint32_t)ty0 | ((uint32_t)a0 << 8) | ((uint32_t)na << 16) | ((uint32_t)nc << 24);
    }
    // start of each tile's run for the first unit (the scan's barriers also
    // order the tables above before their reads)
    uint32_t start;
    {
        const uint32_t c = t < g.tiles ? btot[(size_t)v * 256 + t] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(c, total, s_w);
        start = pbase[v] + ex;
        if (t < g.tiles) {
            const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
            int before = 0;
            for (int x = 0; x <= tx; x++) before += s_d[ty * dw + x];
            start += bcnt[((size_t)v * cpv + j) * 256 + t] + (uint32_t)before;
        }
    }
    const uint32_t seg_end = pbase[v] + pcount[v];
    for (uint32_t uk = ua; uk < ub; uk++) {   // uniform
        const uint32_t s0 = uk * BIN_WIN, s1 = min(pj, s0 + (uint32_t)BIN_WIN);
        // (the previous unit's scatter has read the starts)
        __syncthreads();
        if (t < BIN_WIN / 32) s_mark[t] = 0;
#pragma unroll
        for (int ww = 0; ww < 4; ww++) s_wc[ww][t] = 0;
        __syncthreads();
        // the entry holding slot s0, and a mark where each later entry starts
        for (uint32_t e = ea + t; e <= eb; e += BLOCK) {
            const uint32_t o0 = s_off[e], o1 = e + 1 < nvis ? s_off[e + 1] : pj;
            if (o0 <= s0 && s0 < o1) s_ej = e;
            if (s0 < o0 && o0 < s1) atomicOr(&s_mark[(o0 - s0) >> 5], 1u << ((o0 - s0) & 31));
        }
        __syncthreads();
        if (t < BIN_WIN / 32) {   // marks before each word: one wave's scan of the 64 word counts
            const uint32_t c1 = (uint32_t)__popc(s_mark[t]);
            uint32_t x = c1;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(x, off);
                if (t >= off) x += y;
            }
            s_mpre[t] = x - c1;
        }
        __syncthreads();
        const uint32_t ej = s_ej;
        // wave w takes slots [wb, wb + per) of the unit, 64 per round
        const uint32_t n = s1 - s0;
        const uint32_t per = (n + 4 * 64 - 1) / (4 * 64) * 64;
        const uint32_t wb = (uint32_t)w * per;
        uint32_t key[BIN_WIN / 256], rk[BIN_WIN / 256], val[BIN_WIN / 256];
#pragma unroll
        for (int r = 0; r < BIN_WIN / 256; r++) {
            key[r] = 0xFFFFFFFFu;
            rk[r] = 0;
            val[r] = 0;
            if ((uint32_t)r * 64 >= per) continue;   // uniform
            const uint32_t i = wb + (uint32_t)r * 64 + lane;
            const bool valid = i < n;
            uint32_t d = 0;
            if (valid) {
                // entry: the one holding s0 plus the marks at or before slot i
                const uint32_t wd = i >> 5;
                const uint32_t e = ej + s_mpre[wd] + (uint32_t)__popc(s_mark[wd] & ((2u << (i & 31)) - 1u));
                const uint32_t rc = s_rect[e];
                const int nc = (int)(rc >> 24), na = (int)((rc >> 16) & 255u);
                const int kk = (int)(s0 + i - s_off[e]);
                // kk / nc through the reciprocal (exact after the correction: kk < 2^24)
                int rw = (int)((float)kk * __builtin_amdgcn_rcpf((float)nc));
                int cc = kk - rw * nc;
                if (cc < 0) {
                    rw--;
                    cc += nc;
                } else if (cc >= nc) {
                    rw++;
                    cc -= nc;
                }
                const int ty = (int)(rc & 255u) + rw;
                const int tx = cc < na ? (int)((rc >> 8) & 255u) + cc : cc - na;   // the second run starts at column 0
                d = (uint32_t)(ty * g.tiles_x + tx);
                key[r] = d;
                val[r] = (uint32_t)(row + e);
            }
            const uint64_t m = match_key8(d, __ballot(valid));
            const uint32_t below = (uint32_t)count_below(m);
            const uint32_t before = valid ? s_wc[w][d] : 0u;
            rk[r] = before + below;
            if (valid && below == 0) s_wc[w][d] = before + (uint32_t)__popcll(m);
        }
        __syncthreads();
        {
            const uint32_t c0w = s_wc[0][t], c1w = s_wc[1][t], c2w = s_wc[2][t], c3w = s_wc[3][t];
            s_wc[0][t] = start;
            s_wc[1][t] = start + c0w;
            s_wc[2][t] = start + c0w + c1w;
            s_wc[3][t] = start + c0w + c1w + c2w;
            start += c0w + c1w + c2w + c3w;   // the next unit's start
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < BIN_WIN / 256; r++)
            if (key[r] != 0xFFFFFFFFu) {
                const uint32_t o = s_wc[w][key[r]] + rk[r];
                if (o < seg_end) pval[o] = val[r];
            }
    }
}

// One workgroup per view: the view's per-tile list lengths (the direct
// binning's totals, or the pair sort's digit totals); their exclusive scan
// from the view's segment start gives the lists' positions.  A view without
// pairs has empty lists (its totals are not read: they are not written when
// a render has no pairs at all).  Also the view's tiles ordered by list
// length, longest first (ties by tile index): the blend starts the longest
// lists of every view first, which shortens the tail of its grid.
__device__ __forceinline__ void ranges_of_view(int v, const uint32_t *__restrict__ hist,
                                               const uint32_t *__restrict__ pbase,
                                               const uint32_t *__restrict__ pcount, int tiles,
                                               uint2 *__restrict__ ranges, uint32_t *__restrict__ torder)
{
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_c[BLOCK];
    const int t = threadIdx.x;
    const uint32_t c = pcount[v] ? hist[(size_t)v * 256 + t] : 0u;
    s_c[t] = c;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(c, tot, s_w);
    if (t < tiles) {
        const uint32_t s0 = pbase[v] + ex;
        ranges[(size_t)v * tiles + t] = c ? make_uint2(s0, s0 + c) : make_uint2(0u, 0u);
        int rank = 0;
        for (int u = 0; u < tiles; u++) {
            const uint32_t cu = s_c[u];
            rank += (cu > c || (cu == c && u < t)) ? 1 : 0;
        }
        torder[(size_t)v * tiles + rank] = (uint32_t)t;
    }
}

// [start, end) of each (view, tile) list in the sorted pair array; a view's
// pairs are the first pcount entries of its segment (the rest is not written)
__global__ __launch_bounds__(BLOCK) void k_ranges(const uint32_t *__restrict__ skey, uint32_t Dpad,
                                                  const int4 *__restrict__ segtab,
                                                  const uint32_t *__restrict__ pcount, int tiles,
                                                  uint2 *__restrict__ ranges)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= Dpad) return;
    const int4 e = segtab[i / SORT_TILE];
    const uint32_t first = (uint32_t)e.x * SORT_TILE, end = first + pcount[e.z];
    if (i >= end) return;
    const uint32_t key = skey[i];
    if (key >= (uint32_t)tiles) return;
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
    const int4 vi = vinfo[lo];   // (first receiver, receivers, visible, takes the weights pass)
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

// The tile ranges (one workgroup per view) and the MLP work
// items (the workgroups after them) in one launch; also clears a buffer.
__global__ __launch_bounds__(BLOCK) void k_ranges_items(const uint32_t *__restrict__ hist,
                                                        const uint32_t *__restrict__ pbase,
                                                        const uint32_t *__restrict__ pcount, int tiles,
                                                        uint2 *__restrict__ ranges, uint32_t *__restrict__ torder,
                                                        const uint32_t *__restrict__ item_off,
                                                        const int4 *__restrict__ vinfo, int V, int nitems,
                                                        int4 *__restrict__ items, uint32_t *__restrict__ z,
                                                        size_t nz)
{
    // clears z (the position-block marks of the radiance prefix path)
    for (size_t k = (size_t)blockIdx.x * BLOCK + threadIdx.x; k < nz; k += (size_t)gridDim.x * BLOCK) z[k] = 0u;
    if ((int)blockIdx.x < V) {
        ranges_of_view(blockIdx.x, hist, pbase, pcount, tiles, ranges, torder);
        return;
    }
    const int i = ((int)blockIdx.x - V) * BLOCK + threadIdx.x;
    if (i < nitems) items[i] = make_item(i, item_off, vinfo, V);
}

// Gaussian ("local") term of layer 1: L_k = W1[:, 36:] f_k + b1, in hid_pos
// order, on FP32 MFMA (v_mfma_f32_32x32x2f32).  One wave per 32 Gaussians:
// D (64 hidden x 32 Gaussians) = W1f (64 x 32 features) F^T, with feature
// c = q + 16 h at step q in lane half h, so each lane loads 16 contiguous
// features of its Gaussian; the accumulator register r of block mb in lane
// half h is hidden unit 32 mb + 8 (r / 4) + 4 h + r % 4, stored at position
// 32 h + 16 mb + r of the row, so each lane writes 32 contiguous floats.
// Waves are persistent; W1f and b1 stay in registers.
__global__ __launch_bounds__(BLOCK) void k_mlp_local(const float *__restrict__ W1, const float *__restrict__ b1,
                                                     const float *__restrict__ feat, int64_t K,
                                                     float *__restrict__ Lp, unsigned *__restrict__ amax)
{
    const int lane = threadIdx.x & 63, h = lane >> 5, g = lane & 31;
    float wa[2][16], bias[2][16];
#pragma unroll
    for (int mb = 0; mb < 2; mb++)
#pragma unroll
        for (int q = 0; q < 16; q++) {
            wa[mb][q] = W1[(32 * mb + g) * MLP_IN + ENC + q + 16 * h];
            bias[mb][q] = b1[32 * mb + 8 * (q >> 2) + 4 * h + (q & 3)];
        }
    const int64_t ngroups = (K + 31) / 32;
    float m = 0.f;
    for (int64_t grp = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); grp < ngroups;
         grp += (int64_t)gridDim.x * (BLOCK / 64)) {
        const int64_t k = grp * 32 + g;
        const bool valid = k < K;
        float f[16];
        {
            const float4 *src = reinterpret_cast<const float4 *>(feat + (size_t)min(k, K - 1) * FEAT + 16 * h);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float4 x = src[q];
                f[4 * q] = x.x; f[4 * q + 1] = x.y; f[4 * q + 2] = x.z; f[4 * q + 3] = x.w;
            }
        }
        floatx16 acc0, acc1;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            acc0[r] = bias[0][r];
            acc1[r] = bias[1][r];
        }
#pragma unroll
        for (int q = 0; q < 16; q++) {
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(wa[0][q], f[q], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(wa[1][q], f[q], acc1, 0, 0, 0);
        }
        if (valid) {
            float4 *dst = reinterpret_cast<float4 *>(Lp + (size_t)k * HID + 32 * h);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                dst[q] = make_float4(acc0[4 * q], acc0[4 * q + 1], acc0[4 * q + 2], acc0[4 * q + 3]);
                dst[4 + q] = make_float4(acc1[4 * q], acc1[4 * q + 1], acc1[4 * q + 2], acc1[4 * q + 3]);
            }
#pragma unroll
            for (int r = 0; r < 16; r++) m = fmaxf(m, fmaxf(fabsf(acc0[r]), fabsf(acc1[r])));
        }
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
                                                     float2 *__restrict__ rad, const int *__restrict__ nlive)
{
    if (nlive) nitems = min(nitems, *nlive);
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
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// Split two FP32 values into FP16 (hi, lo) pairs, v = hi + lo: hi is v with
// its 13 low mantissa bits cleared, exactly an FP16 value while |v| is in the
// FP16 normal range (below it the dropped part is under 2^-24 in absolute
// value), lo = v - hi is exact in FP32 and below one FP16 ulp of v, so its
// rounding toward zero costs at most 2^-21 |v|.  Two packing conversions
// for the pair.
__device__ __forceinline__ void split2(float a, float b, half2v &hi, half2v &lo)
{
    const float ha = __uint_as_float(__float_as_uint(a) & 0xFFFFE000u);
    const float hb = __uint_as_float(__float_as_uint(b) & 0xFFFFE000u);
    hi = (half2v)__builtin_amdgcn_cvt_pkrtz(ha, hb);
    lo = (half2v)__builtin_amdgcn_cvt_pkrtz(a - ha, b - hb);
}

__device__ __forceinline__ half8 cat4(const half2v &a, const half2v &b, const half2v &c, const half2v &d)
{
    return __builtin_shufflevector(__builtin_shufflevector(a, b, 0, 1, 2, 3), __builtin_shufflevector(c, d, 0, 1, 2, 3),
                                   0, 1, 2, 3, 4, 5, 6, 7);
}

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

// the 16 features of one lane's Gaussian that its lane half feeds to the
// layer-1 MFMA: f[8 h .. 8 h + 7] and f[16 + 8 h .. 16 + 8 h + 7]
__device__ __forceinline__ void load_feat16(const float *__restrict__ feat, size_t k, int h, float (&f)[16])
{
    const float4 *a = reinterpret_cast<const float4 *>(feat + k * FEAT + 8 * h);
    const float4 *b = reinterpret_cast<const float4 *>(feat + k * FEAT + 16 + 8 * h);
    const float4 x0 = a[0], x1 = a[1], y0 = b[0], y1 = b[1];
    f[0] = x0.x; f[1] = x0.y; f[2] = x0.z; f[3] = x0.w; f[4] = x1.x; f[5] = x1.y; f[6] = x1.z; f[7] = x1.w;
    f[8] = y0.x; f[9] = y0.y; f[10] = y0.z; f[11] = y0.w; f[12] = y1.x; f[13] = y1.y; f[14] = y1.z; f[15] = y1.w;
}

// Layer-1 term of the 32 Gaussians of a work item, L = W1[:, 36:] f + b1, on
// FP16 MFMA in split precision (as layer 2): A = W1's feature block * 2^w1exp
// from LDS, B = the features; the accumulator rows of lane half h are hidden
// units hid_of(h, t), so L lands in the order the activations are built in.
__device__ __forceinline__ void local_term(const float (&f)[16], const half8 *s_w1h, const float4 *s_b1, int lane,
                                           int h, int z0, float unscale, float (&l)[32])
{
    half8 fh[2], fl[2];
#pragma unroll
    for (int q = 0; q < 2; q++) {
        half2v hh[4], ll[4];
#pragma unroll
        for (int i = 0; i < 4; i++) split2(f[8 * q + 2 * i], f[8 * q + 2 * i + 1], hh[i], ll[i]);
        fh[q] = cat4(hh[0], hh[1], hh[2], hh[3]);
        fl[q] = cat4(ll[0], ll[1], ll[2], ll[3]);
    }
    const float4 *b1h = s_b1 + h * 8 + z0;
    floatx16 L0, L1;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const float4 u = b1h[r], w = b1h[4 + r];
        L0[4 * r] = u.x; L0[4 * r + 1] = u.y; L0[4 * r + 2] = u.z; L0[4 * r + 3] = u.w;
        L1[4 * r] = w.x; L1[4 * r + 1] = w.y; L1[4 * r + 2] = w.z; L1[4 * r + 3] = w.w;
    }
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const half8 h0 = s_w1h[((0 * 2 + 0) * 2 + q) * 64 + lane + z0];
        const half8 h1 = s_w1h[((0 * 2 + 1) * 2 + q) * 64 + lane + z0];
        const half8 l0 = s_w1h[((1 * 2 + 0) * 2 + q) * 64 + lane + z0];
        const half8 l1 = s_w1h[((1 * 2 + 1) * 2 + q) * 64 + lane + z0];
        L0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(l0, fh[q], L0, 0, 0, 0);
        L1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(l1, fh[q], L1, 0, 0, 0);
        L0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(h0, fl[q], L0, 0, 0, 0);
        L1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(h1, fl[q], L1, 0, 0, 0);
        L0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(h0, fh[q], L0, 0, 0, 0);
        L1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(h1, fh[q], L1, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 16; t++) {
        l[t] = L0[t] * unscale;
        l[16 + t] = L1[t] * unscale;
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
template <bool SCALED, bool FUSED>
__device__ __forceinline__ void mlp_pairs_walk(const float *__restrict__ Lp, const float *__restrict__ feat,
                                               const float *__restrict__ Gp, const half8 *s_w2h,
                                               const float4 *s_b2, const float4 *s_w3, const half8 *s_w1h,
                                               const float4 *s_b1, float l1unscale, float b30, float b31, float sx,
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
    float l[32], g[32], fv[16];
    const int64_t k0 = min((int64_t)order[(size_t)dc.x * Kp + dc.y + pl], K - 1);
    if (FUSED) load_feat16(feat, (size_t)k0, h, fv);
    else load_half_row(Lp, (size_t)k0, h, l);
    load_half_row(Gp, (size_t)dc.z, h, g);
    for (int n = 0; n < nmine; n++) {
        if (FUSED) {
            int z1 = 0;
            asm volatile("" : "+v"(z1));
            local_term(fv, s_w1h, s_b1, lane, h, z1, l1unscale, l);
        }
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
            for (int q = 0; q < 4; q++) {
                half2v hh[4], ll[4];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int t = 8 * q + 2 * i;
                    float v0 = fmaxf(l[t] + g[t], 0.f), v1 = fmaxf(l[t + 1] + g[t + 1], 0.f);
                    if (SCALED) {
                        v0 *= sx;
                        v1 *= sx;
                    }
                    split2(v0, v1, hh[i], ll[i]);
                }
                bh[q] = cat4(hh[0], hh[1], hh[2], hh[3]);
                bl[q] = cat4(ll[0], ll[1], ll[2], ll[3]);
            }
            const bool last = jj + 1 == nj;
            if (last && more) {
                if (FUSED) load_feat16(feat, (size_t)min((int64_t)kA, K - 1), h, fv);
                else load_half_row(Lp, (size_t)min((int64_t)kA, K - 1), h, l);
            }
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

// FUSED: the Gaussians' layer-1 term is computed here from their features
// (half the bytes of a stored term per pair) and bounded by lbound from the
// host; otherwise it is read from Lp and bounded by its tracked maximum.
template <bool FUSED>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_mlp_pairs(
    const float *__restrict__ Lp, const float *__restrict__ feat,
                                                     const float *__restrict__ Gp, const half8 *__restrict__ w2h,
                                                     const float4 *__restrict__ tab, const float *__restrict__ b3,
                                                     const half8 *__restrict__ w1h, const float *__restrict__ b1tab,
                                                     float l1unscale, float lbound,
                                                     const uint32_t *__restrict__ order,
                                                     const int4 *__restrict__ items, int nitems, int64_t Kp,
                                                     int64_t K, const unsigned *__restrict__ amax,
                                                     float2 *__restrict__ rad, const int *__restrict__ nlive)
{
    if (nlive) nitems = min(nitems, *nlive);
    __shared__ half8 s_w1h[FUSED ? 8 * 64 : 1];
    __shared__ float4 s_b1[FUSED ? 2 * 8 : 1];
    if (FUSED) {
        for (int i = threadIdx.x; i < 8 * 64; i += BLOCK) s_w1h[i] = w1h[i];
        if (threadIdx.x < 64) reinterpret_cast<float *>(s_b1)[threadIdx.x] = b1tab[threadIdx.x];
    }
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
    // largest layer-1 term magnitudes (receivers, and Gaussians unless
    // bounded by the host), spread over 64 slots each
    unsigned mg = amax[lane], ml = FUSED ? 0u : amax[64 + lane];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        mg = max(mg, (unsigned)__shfl_xor((int)mg, o));
        ml = max(ml, (unsigned)__shfl_xor((int)ml, o));
    }
    const float bound = __uint_as_float(mg) + (FUSED ? lbound : __uint_as_float(ml));
    if (bound < 32768.f) {
        mlp_pairs_walk<false, FUSED>(Lp, feat, Gp, s_w2h, s_b2, s_w3, s_w1h, s_b1, l1unscale, b30, b31, 1.f, order,
                                     items, nitems, Kp, K, rad);
    } else {
        int e = 0;
        frexpf(bound, &e);   // bound < 2^e
        const float sx = (e > 15 && e < 128) ? ldexpf(1.f, 15 - e) : 1.f;
        mlp_pairs_walk<true, FUSED>(Lp, feat, Gp, s_w2h, s_b2, s_w3, s_w1h, s_b1, l1unscale, b30, b31, sx, order,
                                    items, nitems, Kp, K, rad);
    }
}

// ----------------------------------------------------------------------------
// Stage 3: front-to-back compositing.  One workgroup per (tile, chunk of R
// receivers of one view); one pixel per thread, each wave an 8 x 8 sub-tile.
// Batches of 256 list entries are staged in LDS; while staging, each entry's
// conservative support box is tested against the four sub-tiles and a
// ballot/prefix pass builds, per wave, the ordered list of entries that can
// reach it, so a wave walks only those.  Every lane keeps its own
// transmittance; a wave stops once all its lanes have terminated and the
// workgroup stops staging once all its waves have.
//
// Two kernels.  With one receiver per workgroup (RX mode, and TX chunks of one
// receiver) the staged form is per (wave, entry), so the walk needs no
// indirection: with
// (X, Y) a pixel's offset from its sub-tile's centre (lane constants, halves
// of odd integers) and (du0, dv0) the entry's centre-to-sub-tile-centre offset,
// the blend exponent (the log2 weight, Sec. 4.3 Eq. for alpha) is the quadratic
//   E = E0 + gx X + gy Y + a X^2 + b XY + c Y^2,
//   E0 = du0 (a du0 + b dv0) + c dv0^2 + log2 o,  gx = 2 a du0 + b dv0,
//   gy = b du0 + 2 c dv0,
// evaluated in five FMAs.  A batch holding an entry that spans more than half
// the azimuth circle keeps (du0, dv0, log2 o) instead and wraps each pixel's
// azimuth offset into [-W/2, W/2).  Record (32 B): (E0 | du0, gx | dv0,
// gy | log2 o, a), (b, c, radiance).  With several receivers per workgroup
// (TX chunks) the walk is bound by broadcasting their radiance from LDS, and
// the shared per-entry form below serves better (k_blend_fwd_multi).

// list entries a wave scans per step (one per lane)
constexpr int BW_CH = 64;

// Far entries of the radiance prefix path: a lane that composites an entry
// past the prefix (its radiance not yet evaluated) records (T w, sorted
// position) so its contribution can be added, in list order, once the
// radiance exists; up to FAR_REC per pixel, more sends the view to a full
// second blend.
constexpr int FAR_REC = FAR_RECORDS;
struct FarState {
    uint2 *rec;      // per (view, pixel): FAR_REC records (bits of T w, sorted position)
    uint8_t *cnt;    // per (view, pixel): records made (saturating at 255)
    uint8_t *tile;   // per (view, tile): some pixel made records
    uint8_t *mark;   // per block of MLP_PAIRS sorted positions: a record points into it
};

// Per wave, the records of the entries of one step of the tile list that can
// reach its sub-tile, in list order (padded with zero-weight records to a
// multiple of 4), their sorted positions and their indices in the tile list.
struct BlendWaveStage {
    float4 q[1][BW_CH + 4][2];           // (E0, gx, gy, a), (b, c, radiance)
    float4 qw[1][BW_CH + 4];             // offset form: (du0, dv0, log2 o, -)
    uint32_t p[1][BW_CH + 4];
    unsigned short idx[1][BW_CH + 4];
    uint32_t wf[1][(BW_CH + 4) / 4];     // one byte per entry: it needs the wrapped form
};

// Four entries of one wave's walk, free of branches per entry: an entry below
// the alpha threshold, or met after the lane terminated, gets weight 0, which
// leaves T and the sums unchanged.  WRAP: the offset form, each pixel's
// azimuth offset wrapped into [-W/2, W/2); else the quadratic form.  CLAMP:
// some entry may reach the 0.99 weight cap.  SAVE: track the stop index and
// the composited count (saved states and statistics only).  DETECT: record
// every entry at index i_far or later that the lane composites (FarState).
template <bool SAVE, bool WRAP, bool CLAMP, bool DETECT>
__device__ __forceinline__ void blend_group4(const BlendWaveStage &st, int wv, int i0, int n, float X, float Y,
                                             float XX, float XY, float YY, float Wf, float halfW, float &T,
                                             float2 &acc, int &last, uint32_t &ncomp, uint32_t &neval,
                                             uint32_t &nslot, bool &done, int i_far, uint2 *myrec, int *fcount,
                                             uint8_t *mark)
{
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int i = i0 + k;
        if (SAVE) {
            const bool real = i < n;
            neval += (real && !done) ? 1u : 0u;
            nslot += real ? 1u : 0u;
        }
        const float4 q0 = st.q[wv][i][0];
        const float4 q1 = st.q[wv][i][1];
        float ex;
        if (WRAP) {
            const float4 qw = st.qw[wv][i];
            float du = qw.x + X;
            du = du >= halfW ? du - Wf : du;
            du = du < -halfW ? du + Wf : du;
            const float dv = qw.y + Y;
            ex = fmaf(du, fmaf(q0.w, du, q1.x * dv), fmaf(q1.y * dv, dv, qw.z));
        } else {
            ex = fmaf(q1.y, YY, fmaf(q1.x, XY, fmaf(q0.w, XX, fmaf(q0.z, Y, fmaf(q0.y, X, q0.x)))));
        }
        // (without CLAMP no entry of the list has log2 o >= LOG2_W_MAX, so the
        // weight is below the cap everywhere)
        float w = __builtin_amdgcn_exp2f(ex);
        if (CLAMP) w = fminf(W_MAX, w);
        const bool inc = !done && w >= ALPHA_MIN;
        w = inc ? w : 0.f;
        const float tw = T * w;
        acc.x = fmaf(tw, q1.z, acc.x);
        acc.y = fmaf(tw, q1.w, acc.y);
        T = T - tw;
        if (SAVE) {
            last = inc ? (int)st.idx[wv][i] + 1 : last;
            ncomp += inc ? 1u : 0u;
        }
        if (DETECT && inc && i >= i_far) {
            if (*fcount < FAR_REC && myrec) {
                const uint32_t pe = st.p[wv][i];
                myrec[*fcount] = make_uint2(__float_as_uint(tw), pe);
                mark[pe / MLP_PAIRS] = 1;
            }
            ++*fcount;
        }
        done = done || T < T_EPS;
    }
}

// One wave's walk over its staged records (n real ones, padded to a multiple
// of 4), four entries in flight.  MIXED: some entry needs the wrapped form
// (bit i of wmask for record i); each group of four that holds one is
// evaluated in the offset form, the others in the quadratic form (a branch
// uniform across the wave).
template <bool SAVE, bool MIXED, bool CLAMP, bool DETECT = false>
__device__ __forceinline__ void blend_walk1(const BlendWaveStage &st, int wv, int n, uint64_t wmask, float X, float Y,
                                            float XX, float XY, float YY, float Wf, float halfW, float &T,
                                            float2 &acc, int &last, uint32_t &ncomp, uint32_t &neval,
                                            uint32_t &nslot, bool &done, int i_begin = 0, int i_far = 0,
                                            uint2 *myrec = nullptr, int *fcount = nullptr, uint8_t *mark = nullptr)
{
    for (int i0 = i_begin; i0 < n; i0 += 4) {
        const bool wrap = MIXED && ((wmask >> i0) & 0xFull) != 0;
        if (wrap)
            blend_group4<SAVE, true, CLAMP, DETECT>(st, wv, i0, n, X, Y, XX, XY, YY, Wf, halfW, T, acc, last, ncomp,
                                                    neval, nslot, done, i_far, myrec, fcount, mark);
        else
            blend_group4<SAVE, false, CLAMP, DETECT>(st, wv, i0, n, X, Y, XX, XY, YY, Wf, halfW, T, acc, last,
                                                     ncomp, neval, nslot, done, i_far, myrec, fcount, mark);
        if (__all(done)) break;
    }
}

template <bool SAVE, bool MIXED, bool CLAMP>
__device__ __forceinline__ void blend_walk1_far(const BlendWaveStage &st, int wv, int n, uint64_t wmask, int i_far, float X,
                                                float Y,
                                                float XX, float XY, float YY, float Wf, float halfW, float &T,
                                                float2 &acc, int &last, uint32_t &ncomp, uint32_t &neval,
                                                uint32_t &nslot, bool &done, uint2 *myrec, int *fcount, uint8_t *mark)
{
    // entries below the position prefix first (the tile list is in depth
    // order), then the rest with the far-entry records
    const int i4 = i_far & ~3;
    blend_walk1<SAVE, MIXED, CLAMP>(st, wv, min(n, i4), wmask, X, Y, XX, XY, YY, Wf, halfW, T, acc, last, ncomp, neval,
                                   nslot, done);
    if (i4 < n && __any(!done))
        blend_walk1<SAVE, MIXED, CLAMP, true>(st, wv, n, wmask, X, Y, XX, XY, YY, Wf, halfW, T, acc, last, ncomp, neval,
                                             nslot, done, i4, i_far, myrec, fcount, mark);
}

// SECOND: the prefix path's second launch (its own instantiation, so that
// profiles tell the two launches apart).
//
// One wave per workgroup, each an 8 x 8 sub-tile of a tile (four workgroups
// per tile and receiver chunk), so a wave whose pixels stop early leaves at
// once: per step, lane l takes entry l of the next 64 of the tile
// list and tests the entry's binning box (the box the tile binning used, so
// every pixel the entry can reach lies in it) against the wave's sub-tile;
// the lanes of the entries that hit build their records (exponent as the
// quadratic around the sub-tile centre, or the wrapped form when an entry
// of the step spans nearly the whole azimuth circle and is centred near the
// sub-tile's antipode, where pixel offsets cross the seam) into the wave's LDS
// slice in list order (ballot and lane count), and the wave walks them.  A
// wave stops at the first step after all its lanes terminated.
constexpr int BLEND1_THREADS = 64;

// (seven waves per SIMD; six for the saving instantiation, whose counters
// would not fit in registers)
template <bool SAVE, bool SECOND = false>
__global__ __launch_bounds__(BLEND1_THREADS) __attribute__((amdgpu_waves_per_eu(SAVE ? 6 : 7, 8))) void k_blend_fwd1(const float4 *__restrict__ srec,
                                                      const float4 *__restrict__ sbox,
                                                      const uint32_t *__restrict__ pval,
                                                      const uint2 *__restrict__ ranges,
                                                      const float2 *__restrict__ rad,
                                                      const int4 *__restrict__ chunks, int64_t Kp, DevGrid g,
                                                      float *__restrict__ C, float *__restrict__ Tfin,
                                                      int *__restrict__ nlast, float *__restrict__ part,
                                                      unsigned long long *__restrict__ stats,
                                                      const uint32_t *__restrict__ torder,
                                                      uint32_t *__restrict__ vflag, uint32_t mpos, FarState fs)
{
    constexpr bool redo = SECOND;
    __shared__ BlendWaveStage st;

    // grid: (chunk, 4 x rank of the tile in its view's longest-first order +
    // sub-tile)
    const int4 ch = chunks[blockIdx.x];
    const int sub = (int)(blockIdx.y & 3u), rank = (int)(blockIdx.y >> 2);
    const int tile = torder ? (int)torder[(size_t)ch.x * g.tiles + rank] : rank;
    const size_t tsub = ((size_t)ch.x * g.tiles + tile) * 4 + sub;   // (view, tile, sub-tile)
    // second launch of the prefix path: blend views that overflowed their
    // records again, add the recorded far entries in sub-tiles that have
    // some, nothing elsewhere
    bool deferred = false;
    if (redo) {
        if (!(vflag[ch.x] & 4u)) {
            if (!fs.tile[tsub]) return;
            deferred = true;
        }
    }
    const int view = ch.x, j0 = ch.y, nrx = ch.z, tslot = ch.w;
    const int ty = tile / g.tiles_x, tx = tile - ty * g.tiles_x;
    const int lane = threadIdx.x, wv = 0;
    const int row = ty * TILE + 8 * (sub >> 1) + (lane >> 3), col = tx * TILE + 8 * (sub & 1) + (lane & 7);
    const bool inside = row < g.H && col < g.W;
    const float X = (float)(lane & 7) - 3.5f, Y = (float)(lane >> 3) - 3.5f;
    const float XX = X * X, XY = X * Y, YY = Y * Y;
    const float Wf = (float)g.W, halfW = 0.5f * (float)g.W, invW = 1.0f / (float)g.W;
    const uint2 rg = ranges[(size_t)view * g.tiles + tile];
    const int64_t view_end = ((int64_t)view + 1) * Kp;
    // this wave's sub-tile: first column and row, centre
    const float cl = (float)(tx * TILE + 8 * (sub & 1)), rl = (float)(ty * TILE + 8 * (sub >> 1));
    const float colc = cl + 3.5f, rowc = rl + 3.5f;
    const float allcols = 0.5f * (float)(g.W - TILE - 2);   // a box this wide takes every tile column

    float T = 1.f;
    float2 acc = make_float2(0.f, 0.f);
    int last = 0;
    uint32_t ncomp = 0, neval = 0, nslot = 0;   // composited / evaluated while active / walked (SAVE)
    bool done = !inside;
    const size_t P = (size_t)g.H * g.W;
    const size_t pix = (size_t)row * g.W + col;
    int fcount = 0;
    uint2 *myrec = (inside && mpos != 0xFFFFFFFFu) ? fs.rec + ((size_t)view * P + pix) * FAR_REC : nullptr;

    if (deferred) {
        // the first pass's sum, then its recorded entries in list order with
        // their radiance: the same operations, in the same order, as one pass
        if (inside && nrx > 0) {
            acc.x = C[((size_t)j0 * 2) * P + pix];
            acc.y = C[((size_t)j0 * 2 + 1) * P + pix];
            const size_t q = (size_t)view * P + pix;
            const int n = min((int)fs.cnt[q], FAR_REC);
            for (int k = 0; k < n; k++) {
                const uint2 rc = fs.rec[q * FAR_REC + k];
                const float tw = __uint_as_float(rc.x);
                const int64_t s = (int64_t)rc.y - (int64_t)view * Kp;
                const float2 sv = rad[(size_t)j0 * Kp + s];
                acc.x = fmaf(tw, sv.x, acc.x);
                acc.y = fmaf(tw, sv.y, acc.y);
            }
        }
    }
    for (uint32_t base = rg.x; !deferred && base < rg.y; base += BW_CH) {
        if (__all(done)) break;   // uniform across the wave
        const uint32_t i = base + (uint32_t)lane;
        uint32_t p = 0;
        bool hit = false, wide = false;
        if (i < rg.y) {
            p = min(pval[i], (uint32_t)(view_end - 1));
            const float4 b = sbox[p];   // (u, v, padded half-extents)
            // the azimuth representative nearest the sub-tile's centre: no
            // other one can reach the sub-tile unless the box spans nearly
            // the whole circle (then it takes every column)
            const float u = fmaf(rintf((colc - b.x) * invW), Wf, b.x);
            const bool colhit = b.z >= allcols || (u + b.z >= cl && u - b.z <= cl + 7.f);
            const bool rowhit = b.y + b.w >= rl && b.y - b.w <= rl + 7.f;
            hit = colhit && rowhit;
            // pixel offsets (u within 3.5 px of the sub-tile's centre) cross
            // the +-W/2 seam only for a centre within 4 px of the antipode,
            // and matter there only for a box reaching that far: such an
            // entry needs the wrapped form
            wide = fabsf(colc - u) > halfW - 4.0f && b.z > halfW - 5.0f;
        }
        const int64_t s = (int64_t)p - (int64_t)view * Kp;
        const bool nearp = s < (int64_t)mpos;
        const uint64_t hb = __ballot(hit);
        const int n = __popcll(hb);
        if (n == 0) continue;
        const bool anywide = __ballot(hit && wide) != 0;
        const int n_near = __popcll(__ballot(hit && nearp));
        // log2 o of some entry at or above log2 0.99 (the weight cap may apply)
        bool capped = false;
        if (hit) {
            const int pos = count_below(hb);
            float4 r0 = srec[2 * (size_t)p];
            const float4 r1 = srec[2 * (size_t)p + 1];
            const float2 re = nearp ? rad[(size_t)j0 * Kp + s] : make_float2(0.f, 0.f);
            // representative of the azimuth closest to the sub-tile's centre
            r0.x = fmaf(rintf((colc - r0.x) * invW), Wf, r0.x);
            const float a = r1.x, bb = r1.y, c = r1.z;
            const float du0 = (colc - r0.x) - r0.y;
            const float dv0 = (rowc - r0.z) - r0.w;
            const float e0 = fmaf(du0, fmaf(a, du0, bb * dv0), fmaf(c * dv0, dv0, r1.w));
            capped = r1.w >= LOG2_W_MAX;
            st.q[wv][pos][0] = make_float4(e0, fmaf(2.f * a, du0, bb * dv0), fmaf(bb, du0, 2.f * c * dv0), a);
            st.q[wv][pos][1] = make_float4(bb, c, re.x, re.y);
            if (anywide) {
                st.qw[wv][pos] = make_float4(du0, dv0, r1.w, 0.f);
                reinterpret_cast<unsigned char *>(st.wf[wv])[pos] = wide ? 1 : 0;
            }
            st.p[wv][pos] = p;
            if (SAVE) st.idx[wv][pos] = (unsigned short)(i - rg.x);
        }
        const bool clamp = __ballot(capped) != 0;
        // zero-weight padding to a multiple of 4: E = -inf in either form
        // (only the constant term is infinite, so no product of infinity and
        // zero arises)
        const int np = (n + 3) & ~3;
        if (lane >= n && lane < np) {
            st.q[wv][lane][0] = make_float4(-INFINITY, 0.f, 0.f, 0.f);
            st.q[wv][lane][1] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (anywide) {
                st.qw[wv][lane] = make_float4(0.f, 0.f, -INFINITY, 0.f);
                reinterpret_cast<unsigned char *>(st.wf[wv])[lane] = 0;
            }
            st.p[wv][lane] = 0;
            if (SAVE) st.idx[wv][lane] = 0;
        }
        // the wave reads what its own lanes wrote (LDS operations of one wave
        // complete in order)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // records that need the wrapped form, by position
        const uint64_t wmask = anywide ? __ballot(reinterpret_cast<const unsigned char *>(st.wf[wv])[lane] != 0) : 0ull;
        if (n_near < n) {
            if (anywide) {
                if (clamp)
                    blend_walk1_far<SAVE, true, true>(st, wv, n, wmask, n_near, X, Y, XX, XY, YY, Wf, halfW, T, acc, last,
                                                      ncomp, neval, nslot, done, myrec, &fcount, fs.mark);
                else
                    blend_walk1_far<SAVE, true, false>(st, wv, n, wmask, n_near, X, Y, XX, XY, YY, Wf, halfW, T, acc, last,
                                                       ncomp, neval, nslot, done, myrec, &fcount, fs.mark);
            } else {
                if (clamp)
                    blend_walk1_far<SAVE, false, true>(st, wv, n, wmask, n_near, X, Y, XX, XY, YY, Wf, halfW, T, acc, last,
                                                       ncomp, neval, nslot, done, myrec, &fcount, fs.mark);
                else
                    blend_walk1_far<SAVE, false, false>(st, wv, n, wmask, n_near, X, Y, XX, XY, YY, Wf, halfW, T, acc, last,
                                                        ncomp, neval, nslot, done, myrec, &fcount, fs.mark);
            }
        } else if (anywide) {
            if (clamp)
                blend_walk1<SAVE, true, true>(st, wv, n, wmask, X, Y, XX, XY, YY, Wf, halfW, T, acc, last, ncomp, neval,
                                              nslot, done);
            else
                blend_walk1<SAVE, true, false>(st, wv, n, wmask, X, Y, XX, XY, YY, Wf, halfW, T, acc, last, ncomp, neval,
                                               nslot, done);
        } else {
            if (clamp)
                blend_walk1<SAVE, false, true>(st, wv, n, wmask, X, Y, XX, XY, YY, Wf, halfW, T, acc, last, ncomp, neval,
                                               nslot, done);
            else
                blend_walk1<SAVE, false, false>(st, wv, n, wmask, X, Y, XX, XY, YY, Wf, halfW, T, acc, last, ncomp, neval,
                                                nslot, done);
        }
        // the next step overwrites the slice only after this walk read it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (!redo) {
        // a pixel still open at the end of a view's truncated list: the view is redone in full
        if (__any(inside && !done) && lane == 0 && (vflag[view] & 1u)) atomicOr(vflag + view, 2u);
        if (mpos != 0xFFFFFFFFu) {
            // entries past the prefix composited here: records kept (8), or too many (4)
            if (inside) fs.cnt[(size_t)view * P + pix] = (uint8_t)min(fcount, 255);
            const bool any_rec = __any(fcount > 0 && fcount <= FAR_REC);
            const bool any_ovf = __any(fcount > FAR_REC);
            if (lane == 0) {
                fs.tile[tsub] = any_rec ? 1 : 0;
                if (any_ovf || any_rec) atomicOr(vflag + view, any_ovf ? 12u : 8u);
            }
        }
    }

    if (inside && nrx > 0) {
        C[((size_t)j0 * 2) * P + pix] = acc.x;
        C[((size_t)j0 * 2 + 1) * P + pix] = acc.y;
        if (SAVE && tslot >= 0) {
            Tfin[(size_t)tslot * P + pix] = T;
            nlast[(size_t)tslot * P + pix] = last;
        }
    }
    // per-sub-tile partial sums: power, Re, Im (the reduction adds the four
    // sub-tiles of a tile in order, then the tiles)
    {
        // (one explicit FMA, so every instantiation rounds the power alike)
        const float pw = wave_sum_f32(fmaf(acc.x, acc.x, acc.y * acc.y));
        const float sr = wave_sum_f32(acc.x);
        const float si = wave_sum_f32(acc.y);
        if (lane == 0 && nrx > 0) {
            float *pp = part + (((size_t)j0 * g.tiles + tile) * 4 + sub) * 3;
            pp[0] = pw;
            pp[1] = sr;
            pp[2] = si;
        }
    }
    // composited (pixel, entry) pairs: per chunk pixel and per receiver pixel,
    // spread over STAT_SLOTS counters
    if (SAVE) {
        const uint32_t nc = wave_sum_u32(ncomp), ne = wave_sum_u32(neval), ns = wave_sum_u32(nslot);
        if (lane == 0) {
            const unsigned slot = (blockIdx.x + blockIdx.y * gridDim.x) % STAT_SLOTS;
            if (nc) {
                atomicAdd(stats + slot, (unsigned long long)nc);
                atomicAdd(stats + STAT_SLOTS + slot, (unsigned long long)nc * (unsigned long long)nrx);
            }
            if (ns) {
                atomicAdd(stats + 2 * STAT_SLOTS + slot, (unsigned long long)ne);
                atomicAdd(stats + 3 * STAT_SLOTS + slot, (unsigned long long)ns);
            }
        }
    }
}

// Several receivers per workgroup: entries staged once per batch (record,
// batch index lists per wave), radiance of the R receivers in LDS.  One wave's
// walk over its staged list, free of branches per entry: an entry
// below the alpha threshold, or met after the lane terminated, gets weight 0,
// which leaves T and the sums bit-identical to skipping it.  WRAP: some entry of
// the list spans more than half the azimuth circle, so pixel offsets are
// wrapped into [-W/2, W/2) (selects).  SAVE: track the stop index and the
// composited count (saved states and statistics only).  MARK: flag in s_mark
// every entry that some lane composites (the weights-only pass).
template <int R, bool SAVE, bool WRAP, bool MARK = false, bool DETECT = false>
__device__ __forceinline__ void blend_walk_multi(const BlendStage &st, const float2 (*s_rad)[BLOCK], int wv, int n,
                                           int lbase, float colf, float rowf, float Wf, float halfW, float &T,
                                           float2 (&acc)[R], int &last, uint32_t &ncomp, uint32_t &neval,
                                           uint32_t &nslot, bool &done, unsigned char *s_mark = nullptr,
                                           int i_begin = 0, uint2 *myrec = nullptr, int *fcount = nullptr,
                                           uint8_t *mark = nullptr)
{
    for (int i = i_begin; i < n; i++) {
        if (SAVE) {
            neval += done ? 0u : 1u;
            nslot++;
        }
        const int e = st.list[wv][i];
        const float4 r0 = st.r0[e];
        const float4 r1 = st.r1[e];
        float du = (colf - r0.x) - r0.y;
        if (WRAP) {
            du = du >= halfW ? du - Wf : du;
            du = du < -halfW ? du + Wf : du;
        }
        const float dv = (rowf - r0.z) - r0.w;
        float w = fminf(W_MAX, __builtin_amdgcn_exp2f(blend_exponent(du, dv, r1)));
        const bool inc = !done && w >= ALPHA_MIN;
        w = inc ? w : 0.f;
        const float tw = T * w;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const float2 sv = s_rad[r][e];
            acc[r].x = fmaf(tw, sv.x, acc[r].x);
            acc[r].y = fmaf(tw, sv.y, acc[r].y);
        }
        T = T * (1.f - w);
        if (SAVE) {
            last = inc ? lbase + e : last;
            ncomp += inc ? 1u : 0u;
        }
        if (MARK && inc) s_mark[e] = 1;
        if (DETECT && inc) {
            if (*fcount < FAR_REC && myrec) {
                myrec[*fcount] = make_uint2(__float_as_uint(tw), st.p[e]);
                mark[st.p[e] / MLP_PAIRS] = 1;
            }
            ++*fcount;
        }
        done = done || T < T_EPS;
        if ((i & 3) == 3 && __all(done)) break;
    }
}

// MARK (weights-only pass over chunks with no receivers): set live[b] for
// every block b of MLP_PAIRS sorted positions holding an entry that some pixel
// composites; the walk is the colour pass's own, so the decisions are the
// same.  Otherwise, when live is given, positions of unmarked blocks read a
// zero radiance: no pixel composites them, so their weight is zero and the
// sums are unchanged.
template <int R, bool SAVE, bool MARK = false, bool SECOND = false>
__global__ __launch_bounds__(BLOCK) void k_blend_fwd_multi(const float4 *__restrict__ srec,
                                                     const uint32_t *__restrict__ pval,
                                                     const uint2 *__restrict__ ranges,
                                                     const float2 *__restrict__ rad,
                                                     const int4 *__restrict__ chunks, int64_t Kp, DevGrid g,
                                                     float *__restrict__ C, float *__restrict__ Tfin,
                                                     int *__restrict__ nlast, float *__restrict__ part,
                                                     unsigned long long *__restrict__ stats,
                                                     const uint32_t *__restrict__ torder,
                                                     uint8_t *__restrict__ live, uint32_t *__restrict__ vflag,
                                                     uint32_t mpos, FarState fs)
{
    constexpr bool redo = SECOND;
    __shared__ BlendStage st;
    __shared__ float2 s_rad[R][BLOCK];
    __shared__ float s_red[4][R][3];
    __shared__ unsigned char s_mark[MARK ? BLOCK : 1];
    if (MARK) s_mark[threadIdx.x] = 0;

    // grid: (chunk, rank of the tile in its view's longest-first order)
    const int4 ch = chunks[blockIdx.x];
    const int tile = torder ? (int)torder[(size_t)ch.x * g.tiles + blockIdx.y] : (int)blockIdx.y;
    // second launch of the prefix path (see k_blend_fwd1)
    bool deferred = false;
    if (redo) {
        if (!(vflag[ch.x] & 4u)) {
            if (!fs.tile[(size_t)ch.x * g.tiles + tile]) return;
            deferred = true;
        }
    }
    const int view = ch.x, j0 = ch.y, nrx = ch.z, tslot = ch.w;
    const int ty = tile / g.tiles_x, tx = tile - ty * g.tiles_x;
    const int t = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
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
    uint32_t ncomp = 0, neval = 0, nslot = 0;   // composited / evaluated while active / walked (SAVE)
    bool done = !inside;
    const size_t P = (size_t)g.H * g.W;
    const size_t pix = (size_t)row * g.W + col;
    int fcount = 0;
    uint2 *myrec = (!MARK && inside && mpos != 0xFFFFFFFFu) ? fs.rec + ((size_t)view * P + pix) * FAR_REC : nullptr;

    if (deferred && inside) {
        // the first pass's sums, then the view's recorded entries in list order
        // with each receiver's radiance (see k_blend_fwd1)
#pragma unroll
        for (int r = 0; r < R; r++)
            if (r < nrx) {
                acc[r].x = C[((size_t)(j0 + r) * 2) * P + pix];
                acc[r].y = C[((size_t)(j0 + r) * 2 + 1) * P + pix];
            }
        const size_t q = (size_t)view * P + pix;
        const int n = min((int)fs.cnt[q], FAR_REC);
        for (int k = 0; k < n; k++) {
            const uint2 rc = fs.rec[q * FAR_REC + k];
            const float tw = __uint_as_float(rc.x);
            const int64_t s = (int64_t)rc.y - (int64_t)view * Kp;
#pragma unroll
            for (int r = 0; r < R; r++)
                if (r < nrx) {
                    const float2 sv = rad[(size_t)(j0 + r) * Kp + s];
                    acc[r].x = fmaf(tw, sv.x, acc[r].x);
                    acc[r].y = fmaf(tw, sv.y, acc[r].y);
                }
        }
    }
    for (uint32_t base = rg.x; !deferred && base < rg.y; base += BLOCK) {
        const uint32_t cnt = min((uint32_t)BLOCK, rg.y - base);
        __syncthreads();
        uint32_t p = 0;
        bool nearp = true;
        if ((uint32_t)t < cnt) {
            p = min(pval[base + t], (uint32_t)(view_end - 1));
            const int64_t s = max((int64_t)p - (int64_t)view * Kp, (int64_t)0);
            nearp = s < (int64_t)mpos;
            const bool used = MARK || ((live == nullptr || live[p / MLP_PAIRS] != 0) && nearp);
#pragma unroll
            for (int r = 0; r < R; r++)
                s_rad[r][t] = (r < nrx && used) ? rad[(size_t)(j0 + r) * Kp + s] : make_float2(0.f, 0.f);
        }
        stage_batch(st, srec, p, (uint32_t)t < cnt, tx, ty, g, nearp);
        if (__any(!done)) {
            const int n = __builtin_amdgcn_readfirstlane(st.len[wv]);
            const int lbase = (int)(base - rg.x) + 1;
            // list entries below the position prefix come first (the tile list is in depth order)
            const int i_far = __builtin_amdgcn_readfirstlane(st.ncnt[0][wv] + st.ncnt[1][wv] + st.ncnt[2][wv] +
                                                             st.ncnt[3][wv]);
            const bool wrap = __builtin_amdgcn_readfirstlane(st.wrap[wv]) != 0;
            if (wrap)
                blend_walk_multi<R, SAVE, true, MARK>(st, s_rad, wv, i_far, lbase, colf, rowf, Wf, halfW, T, acc,
                                                      last, ncomp, neval, nslot, done, s_mark);
            else
                blend_walk_multi<R, SAVE, false, MARK>(st, s_rad, wv, i_far, lbase, colf, rowf, Wf, halfW, T, acc,
                                                       last, ncomp, neval, nslot, done, s_mark);
            if (i_far < n && __any(!done)) {
                if (wrap)
                    blend_walk_multi<R, SAVE, true, MARK, true>(st, s_rad, wv, n, lbase, colf, rowf, Wf, halfW, T, acc,
                                                                last, ncomp, neval, nslot, done, s_mark, i_far,
                                                                myrec, &fcount, fs.mark);
                else
                    blend_walk_multi<R, SAVE, false, MARK, true>(st, s_rad, wv, n, lbase, colf, rowf, Wf, halfW, T,
                                                                 acc, last, ncomp, neval, nslot, done, s_mark, i_far,
                                                                 myrec, &fcount, fs.mark);
            }
        }
        const int alldone = __syncthreads_and(done ? 1 : 0);
        if (MARK) {
            if ((uint32_t)t < cnt && s_mark[t]) live[st.p[t] / MLP_PAIRS] = 1;
            s_mark[t] = 0;
        }
        if (alldone) break;
    }
    if (MARK) return;
    if (!redo) {
        // a pixel still open at the end of a view's truncated list: the view is redone in full
        if (__syncthreads_or(inside && !done) && t == 0 && (vflag[view] & 1u)) atomicOr(vflag + view, 2u);
        if (mpos != 0xFFFFFFFFu) {
            // entries past the prefix composited here: records kept (8), or too many (4);
            // every chunk of a view walks the same weights and writes the same records
            if (inside) fs.cnt[(size_t)view * P + pix] = (uint8_t)min(fcount, 255);
            const int any_rec = __syncthreads_or(fcount > 0 && fcount <= FAR_REC);
            const int any_ovf = __syncthreads_or(fcount > FAR_REC);
            if (t == 0) {
                fs.tile[(size_t)view * g.tiles + tile] = any_rec ? 1 : 0;
                if (any_ovf || any_rec) atomicOr(vflag + view, any_ovf ? 12u : 8u);
            }
        }
    }

    if (inside) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (r < nrx) {
                C[((size_t)(j0 + r) * 2) * P + pix] = acc[r].x;
                C[((size_t)(j0 + r) * 2 + 1) * P + pix] = acc[r].y;
            }
        }
        if (SAVE && tslot >= 0) {
            Tfin[(size_t)tslot * P + pix] = T;
            nlast[(size_t)tslot * P + pix] = last;
        }
    }
    // per-tile partial sums: power, Re, Im (fixed-order reduction)
#pragma unroll
    for (int r = 0; r < R; r++) {
        const float pw = wave_sum_f32(fmaf(acc[r].x, acc[r].x, acc[r].y * acc[r].y));
        const float sr = wave_sum_f32(acc[r].x);
        const float si = wave_sum_f32(acc[r].y);
        if (lane == 0) {
            s_red[wv][r][0] = pw;
            s_red[wv][r][1] = sr;
            s_red[wv][r][2] = si;
        }
    }
    if (SAVE) {
        const uint32_t nc = wave_sum_u32(ncomp), ne = wave_sum_u32(neval), ns = wave_sum_u32(nslot);
        if (lane == 0) {
            st.wcnt[0][wv] = (int)nc;
            st.wcnt[1][wv] = (int)ne;
            st.wcnt[2][wv] = (int)ns;
        }
    }
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
    if (SAVE && t == 0) {
        const unsigned slot = (blockIdx.x + blockIdx.y * gridDim.x) % STAT_SLOTS;
        unsigned long long n[3];
#pragma unroll
        for (int c = 0; c < 3; c++)
            n[c] = (unsigned long long)st.wcnt[c][0] + st.wcnt[c][1] + st.wcnt[c][2] + st.wcnt[c][3];
        if (n[0]) {
            atomicAdd(stats + slot, n[0]);
            atomicAdd(stats + STAT_SLOTS + slot, n[0] * (unsigned long long)nrx);
        }
        if (n[2]) {
            atomicAdd(stats + 2 * STAT_SLOTS + slot, n[1]);
            atomicAdd(stats + 3 * STAT_SLOTS + slot, n[2]);
        }
    }
}

// one wave per receiver; lanes take tiles in a fixed stride, then a fixed
// butterfly, so the result does not depend on scheduling
// part: per (row, tile) nsub partials of (power, Re, Im), the sub-tiles of a
// tile in order
__global__ __launch_bounds__(BLOCK) void k_reduce_out(const float *__restrict__ part, int N, int tiles, int nsub,
                                                      float *__restrict__ power, float *__restrict__ csum)
{
    const int j = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= N) return;
    double pw = 0, sr = 0, si = 0;
    for (int t = lane; t < tiles; t += 64) {
        const float *p = part + ((size_t)j * tiles + t) * nsub * 3;
        for (int q = 0; q < nsub; q++) {
            pw += p[3 * q];
            sr += p[3 * q + 1];
            si += p[3 * q + 2];
        }
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

bool grow(DevBuf &b, size_t bytes, Allocator *al)
{
    if (bytes == 0) bytes = 256;
    if (b.cap >= bytes && b.al == al) return true;
    release(b);
    if (al && al->base) {   // carved from the fixed region, 256-byte aligned
        const size_t at = (al->used + 255) / 256 * 256;
        if (at > al->cap || bytes > al->cap - at) return false;
        b.p = al->base + at;
        b.cap = bytes;
        b.al = al;
        al->used = at + bytes;
        return true;
    }
    size_t want = bytes + bytes / 4;
    if (al && al->alloc) {
        void *p = al->alloc(want, al->device, al->user);
        if (!p) {
            p = al->alloc(bytes, al->device, al->user);
            want = bytes;
        }
        if (!p) return false;
        b.p = p;
        b.cap = want;
        b.al = al;
        return true;
    }
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
    b.al = al;
    return true;
}

void release(DevBuf &b)
{
    if (b.p) {
        if (b.al && b.al->base) {
            // a carved buffer: the region is rewound as a whole
        } else if (b.al && b.al->free) {
            // the caller's allocator may hand the block out again at once:
            // nothing queued on any stream may still use it
            (void)hipDeviceSynchronize();
            b.al->free(b.p, b.cap, b.al->device, b.al->user);
        } else {
            (void)hipFree(b.p);
        }
    }
    b.p = nullptr;
    b.cap = 0;
    b.al = nullptr;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned blocks = (unsigned)std::min<size_t>(nblk(n), 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(BLOCK), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_project_exports(Workspace &ws, hipStream_t st)
{
    const int V = ws.V;
    const int vchunk = V <= 4 ? 1 : 4;
    if (V == 0 || ws.Kp == 0) return hipSuccess;
    dim3 grid((unsigned)(ws.Kp / BLOCK), (unsigned)((V + vchunk - 1) / vchunk));
    hipLaunchKernelGGL((k_project<true, false>), grid, dim3(BLOCK), 0, st, ws.ggeo.as<GaussGeoPacked>(),
                       ws.qcull.as<float>(), ws.K, ws.Kp, ws.centres.as<float>(), V, vchunk, ws.g, nullptr, nullptr,
                       ws.ext.as<float4>(), ws.rawkey.as<uint32_t>(), ws.opac.as<float>(), nullptr, (size_t)0,
                       nullptr, (size_t)0);
    return hipGetLastError();
}

// scenes from this many (padded) Gaussians take four views per key workgroup
constexpr int64_t KEYS_BIG_SCENE = 1 << 18;

hipError_t launch_project(const Scene &sc, const float *centres, int V, int64_t Kp, const DevGrid &g,
                          Workspace &ws, size_t counter_words, size_t sort_words, hipStream_t st)
{
    if (Kp % (8 * BLOCK) != 0) return hipErrorInvalidValue;
    // (the clears need a grid even without Gaussians)
    const unsigned nb = (unsigned)std::max<int64_t>((sc.K + BLOCK - 1) / BLOCK, 64);
    hipLaunchKernelGGL(k_gauss_prep, dim3(nb), dim3(BLOCK), 0, st, sc.soa.as<float>(), sc.K,
                       ws.ggeo.as<GaussGeoPacked>(), ws.qcull.as<float>(), ws.counters.as<uint32_t>(), counter_words,
                       ws.hist.as<uint32_t>(), sort_words);
    if (V == 0 || Kp == 0) return hipGetLastError();
    const bool wide = (uint64_t)V * (uint64_t)(Kp / (8 * BLOCK)) >= 1024;
    const bool big = wide && V >= 4 && Kp >= KEYS_BIG_SCENE;
    const int per = wide ? 8 : 1, vpw = big ? 4 : 1;
    auto kern = big ? k_keys<8, 4> : wide ? k_keys<8, 1> : k_keys<1, 1>;
    hipLaunchKernelGGL(kern, dim3((unsigned)((uint64_t)((V + vpw - 1) / vpw) * (uint64_t)(Kp / (per * BLOCK)))),
                       dim3(BLOCK), 0, st, ws.ggeo.as<GaussGeoPacked>(), ws.qcull.as<float>(), sc.K, Kp, centres, g,
                       V, ws.skey[0].as<uint32_t>(), ws.hist.as<uint32_t>());
    return hipGetLastError();
}

// the emission's error word, per view the depth sort's kept count (KEPT_STRIDE
// words apart) and per-chunk 64-bit look-back status, after the render
// statistics in the counters buffer (the offset is even, so the status words
// are 8-byte aligned)
uint32_t *emit_words(Workspace &ws)
{
    return ws.counters.as<uint32_t>() + (size_t)4 * ws.V + AMAX_SLOTS + 2 * STAT_WORDS;
}

size_t emit_word_count(int V, int64_t Kp)
{
    return KEPT_STRIDE + (size_t)V * KEPT_STRIDE + 2 * (size_t)V * (size_t)((Kp + BLOCK - 1) / BLOCK);
}

// chunks of 1024 entries (512 threads, 2 per thread) when there are many,
// which amortises each chunk's look-back; 256 (1 per thread) for small
// launches, which keeps the chain of chunks short
void emit1_chunking(Workspace &ws)
{
    const int64_t per_view = std::min<int64_t>(ws.Kp, ws.limit);
    const bool wide = (size_t)ws.V * (size_t)(per_view / (4 * BLOCK)) >= 1024;
    ws.em_chunk = wide ? 4 * BLOCK : BLOCK;
    ws.em_cpv = (int)((per_view + ws.em_chunk - 1) / ws.em_chunk);
    // placement units per workgroup of k_bin_pairs: BIN_GROUP when there are many
    // chunks (fewer set-ups), else one (more workgroups for the heavy chunks)
    ws.bin_group = (size_t)ws.V * (size_t)ws.em_cpv >= 2048 ? BIN_GROUP : 1;
}

size_t bins_bytes(int V, int cpv)
{
    const size_t vc = (size_t)V * cpv;
    return (vc * 256 + vc * 4 + (size_t)V * 256 + (size_t)V + (size_t)V * (cpv + 1)) * 4;
}

namespace {
struct BinPtrs {
    uint32_t *cnt, *tot, *live, *unit;
    uint4 *info;
};
BinPtrs bin_ptrs(Workspace &ws)
{
    BinPtrs b;
    const size_t vc = (size_t)ws.V * ws.em_cpv;
    b.cnt = ws.bins.as<uint32_t>();
    b.info = reinterpret_cast<uint4 *>(b.cnt + vc * 256);
    b.tot = b.cnt + vc * 256 + vc * 4;
    b.live = b.tot + (size_t)ws.V * 256;
    b.unit = b.live + ws.V;
    return b;
}
}  // namespace

hipError_t launch_bin_scan(Workspace &ws, const DevGrid &g, hipStream_t st)
{
    const BinPtrs b = bin_ptrs(ws);
    hipLaunchKernelGGL(k_bin_scan, dim3((unsigned)ws.V), dim3(BLOCK), 0, st, ws.hist.as<uint32_t>(), 4, ws.limit,
                       ws.em_cpv, ws.em_chunk, g.tiles, ws.bin_group, b.info, b.cnt, b.tot, b.live, b.unit);
    return hipGetLastError();
}

hipError_t launch_bin_pairs(Workspace &ws, const DevGrid &g, hipStream_t st)
{
    if (ws.n_emit_chunks == 0) return hipSuccess;
    if (ws.em_chunk > BIN_CHUNK_MAX) return hipErrorInvalidValue;
    const BinPtrs b = bin_ptrs(ws);
    hipLaunchKernelGGL(k_bin_pairs, dim3((unsigned)ws.n_emit_chunks), dim3(BLOCK), 0, st, ws.sbox.as<float4>(),
                       ws.poff.as<uint32_t>(), ws.Kp, g, ws.em_cpv, ws.V, ws.bin_group, ws.d_chunk_off, b.info, b.cnt,
                       b.tot,
                       b.live, b.unit, ws.d_pbase, ws.d_pcount, ws.pval[0].as<uint32_t>());
    return hipGetLastError();
}

hipError_t launch_emit1(const Scene &sc, Workspace &ws, const DevGrid &g, hipStream_t st)
{
    uint32_t *ew = emit_words(ws);
    emit1_chunking(ws);
    const bool wide = ws.em_chunk == 4 * BLOCK;
    const int cpv = ws.em_cpv;
    const BinPtrs b = ws.direct_bins ? bin_ptrs(ws) : BinPtrs{nullptr, nullptr, nullptr, nullptr, nullptr};
    auto kern = wide ? k_emit1<2, 2 * BLOCK> : k_emit1<1, BLOCK>;
    hipLaunchKernelGGL(kern, dim3((unsigned)(ws.V * cpv)), dim3(wide ? 2 * BLOCK : BLOCK), 0, st,
                       ws.ggeo.as<GaussGeoPacked>(), sc.K, ws.Kp, ws.centres_p, g,
                       ws.sval[ws.sorted_buf].as<uint32_t>(), ew + KEPT_STRIDE, cpv, ws.srec.as<float4>(),
                       ws.sbox.as<float4>(), ws.vorder.as<uint32_t>(), ws.poff.as<uint32_t>(),
                       ws.counters.as<unsigned long long>(),
                       reinterpret_cast<unsigned long long *>(ew + KEPT_STRIDE + (size_t)ws.V * KEPT_STRIDE), ew,
                       ws.limit, ws.vflag.as<uint32_t>(), b.cnt, b.info);
    return hipGetLastError();
}

hipError_t launch_emit2(Workspace &ws, const DevGrid &g, size_t sort_words, hipStream_t st)
{
    if (ws.n_emit_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit2, dim3((unsigned)ws.n_emit_chunks), dim3(BLOCK), 0, st, ws.sbox.as<float4>(),
                       ws.poff.as<uint32_t>(), ws.Kp, g, ws.counters.as<unsigned long long>(), ws.d_pbase,
                       ws.d_pcount, ws.d_chunk_off, ws.V, ws.pkey[0].as<uint32_t>(), ws.pval[0].as<uint32_t>(),
                       ws.hist_b.as<uint32_t>(), sort_words);
    return hipGetLastError();
}

hipError_t launch_ranges(Workspace &ws, const DevGrid &g, hipStream_t st)
{
    const size_t nr = (size_t)ws.V * g.tiles;
    ws.items_built = false;
    if (g.tiles <= 255) {
        // one 8-bit pass: ranges straight from the scanned histogram; the MLP
        // work items in the same launch
        const unsigned nbi = ws.use_items ? (unsigned)nblk((size_t)ws.n_items) : 0u;
        if (nbi > 0 && ws.items.cap < (size_t)ws.n_items * 16) return hipErrorInvalidValue;   // not allocated
        // (the list lengths: the direct binning's per-view totals, or the pair sort's digit totals)
        const uint32_t *lens = ws.direct_bins ? bin_ptrs(ws).tot : ws.hist_b.as<uint32_t>();
        // the radiance prefix path's position-block marks are cleared here too
        ws.live_cleared = ws.mpos != 0xFFFFFFFFu;
        hipLaunchKernelGGL(k_ranges_items, dim3((unsigned)ws.V + nbi), dim3(BLOCK), 0, st, lens,
                           ws.d_pbase, ws.d_pcount, g.tiles, ws.ranges.as<uint2>(), ws.torder.as<uint32_t>(),
                           ws.d_item_off, ws.d_vinfo, ws.V, ws.n_items, ws.items.as<int4>(),
                           ws.live_cleared ? ws.live.as<uint32_t>() : nullptr,
                           ws.live_cleared ? (live_count_offset(ws) + 3) / 4 : (size_t)0);
        ws.tiles_ordered = true;
        ws.items_built = nbi > 0;
        return hipGetLastError();
    }
    ws.tiles_ordered = false;
    ws.live_cleared = false;
    hipError_t e = launch_fill_u32(ws.ranges.as<uint32_t>(), 0u, nr * 2, st);
    if (e != hipSuccess || ws.Dpad == 0) return e;
    hipLaunchKernelGGL(k_ranges, dim3(nblk((size_t)ws.Dpad)), dim3(BLOCK), 0, st,
                       ws.pkey[ws.pairs_buf].as<uint32_t>(), (uint32_t)ws.Dpad, ws.d_segtab, ws.d_pcount, g.tiles,
                       ws.ranges.as<uint2>());
    return hipGetLastError();
}

hipError_t launch_rad_direct(const Scene &sc, Workspace &ws, hipStream_t st)
{
    const int64_t n = (int64_t)ws.N * ws.Kp;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rad_direct, dim3(nblk(n)), dim3(BLOCK), 0, st, sc.rad.as<float2>(),
                       ws.vorder.as<uint32_t>(), ws.counters.as<unsigned long long>(),
                       ws.d_rxview, ws.N, ws.Kp, ws.K, ws.rad.as<float2>());
    return hipGetLastError();
}

// render statistics after the activation-bound slots, STAT_SLOTS u64 each:
// composited pairs per chunk pixel, per receiver pixel, entries evaluated by
// lanes still compositing, and wave-entry slots walked (64 per entry a wave walks)
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

// the receivers' layer-1 term (needs no per-render descriptors)
hipError_t launch_mlp_global_term(const Mlp &m, Workspace &ws, hipStream_t st)
{
    const unsigned nbg = (unsigned)nblk((size_t)ws.N * HID);
    if (nbg > 0 && ws.Gp.cap < (size_t)ws.N * HID * 4) return hipErrorInvalidValue;   // not allocated
    if (nbg > 0)
        hipLaunchKernelGGL(k_mlp_global, dim3(nbg), dim3(BLOCK), 0, st, m.raw.as<float>(), ws.rxpos_p, ws.N,
                           ws.Gp.as<float>(), amax_words(ws), (int)nbg, nullptr, nullptr, ws.V, 0, nullptr);
    return hipGetLastError();
}

// the MLP work items, expanded from the per-view offsets
hipError_t launch_mlp_items(Workspace &ws, hipStream_t st)
{
    const unsigned nbi = (unsigned)nblk((size_t)ws.n_items);
    if (nbi > 0 && ws.items.cap < (size_t)ws.n_items * 16) return hipErrorInvalidValue;   // not allocated
    if (nbi > 0)
        hipLaunchKernelGGL(k_mlp_global, dim3(nbi), dim3(BLOCK), 0, st, nullptr, nullptr, 0, nullptr, nullptr, 0,
                           ws.d_item_off, ws.d_vinfo, ws.V, ws.n_items, ws.items.as<int4>());
    return hipGetLastError();
}

hipError_t launch_mlp_local(const Scene &sc, const Mlp &m, Workspace &ws, hipStream_t st)
{
    const float *raw = m.raw.as<float>();
    if (sc.K > 0) {
        const int64_t waves = (sc.K + 31) / 32;
        const unsigned blocks = (unsigned)std::min<int64_t>((waves + 3) / 4, 2048);
        hipLaunchKernelGGL(k_mlp_local, dim3(blocks), dim3(BLOCK), 0, st, raw, raw + HID * MLP_IN,
                           sc.feat.as<float>(), sc.K, ws.Lp.as<float>(), amax_words(ws) + 64);
    }
    return hipGetLastError();
}

bool mlp_fused_ok(const Scene &sc, const Mlp &m)
{
    return !m.fp32 && m.w1_ok && sc.fmax < 32768.f;
}

hipError_t launch_mlp_pairs(const Scene &sc, const Mlp &m, Workspace &ws, hipStream_t st, bool far)
{
    const float *raw = m.raw.as<float>();
    const float *b3 = raw + HID * MLP_IN + HID + HID * HID + HID + 2 * HID;
    // the items: the prefix's (or all), the live ones (lazy TX), or those past the prefix of flagged views
    const int4 *items = far ? ws.items_far.as<int4>() : ws.lazy ? ws.items_live.as<int4>() : ws.items.as<int4>();
    const int *nlive = far ? far_count(ws) : ws.lazy ? live_count(ws) : nullptr;
    const int nmax = far ? ws.n_items_far : ws.n_items;
    if (nmax > 0) {
        const unsigned blocks = (unsigned)std::min((nmax + 3) / 4, 256 * 8);
        if (m.fp32) {
            hipLaunchKernelGGL(k_mlp_pairs_f32, dim3(blocks), dim3(BLOCK), 0, st, ws.Lp.as<float>(),
                               ws.Gp.as<float>(), m.w2a.as<float>(), m.tab.as<float4>(), b3,
                               ws.vorder.as<uint32_t>(), items, nmax, ws.Kp, ws.K,
                               ws.counters.as<unsigned long long>(), ws.rad.as<float2>(), nlive);
        } else if (mlp_fused_ok(sc, m)) {
            // bound of the Gaussians' layer-1 term: per hidden unit
            // sum_c |W1[d, 36 + c]| max|f| + |b1[d]|, rounded up
            double lb = 0.0;
            for (int d = 0; d < HID; d++) lb = std::max(lb, m.w1abs[d] * (double)sc.fmax + m.b1abs[d]);
            const float lbound = (float)(lb * (1.0 + 1e-6)) + 1e-30f;
            hipLaunchKernelGGL(k_mlp_pairs<true>, dim3(blocks), dim3(BLOCK), 0, st, ws.Lp.as<float>(),
                               sc.feat.as<float>(), ws.Gp.as<float>(), m.w2h.as<half8>(), m.tabh.as<float4>(), b3,
                               m.w1h.as<half8>(), m.b1tab.as<float>(), std::ldexp(1.f, -m.w1exp), lbound,
                               ws.vorder.as<uint32_t>(), items, nmax, ws.Kp, ws.K,
                               amax_words(ws), ws.rad.as<float2>(), nlive);
        } else {
            hipLaunchKernelGGL(k_mlp_pairs<false>, dim3(blocks), dim3(BLOCK), 0, st, ws.Lp.as<float>(),
                               sc.feat.as<float>(), ws.Gp.as<float>(), m.w2h.as<half8>(), m.tabh.as<float4>(), b3,
                               m.w1h.as<half8>(), m.b1tab.as<float>(), 1.f, 0.f,
                               ws.vorder.as<uint32_t>(), items, nmax, ws.Kp, ws.K,
                               amax_words(ws), ws.rad.as<float2>(), nlive);
        }
    }
    return hipGetLastError();
}

// sums over a list of MLP work items (view, s0, first receiver, receivers |
// valid positions << 8): items, (receiver, position) pairs, 32-slot pairs
__global__ __launch_bounds__(BLOCK) void k_count_items(const int4 *__restrict__ items, int nmax,
                                                       const int *__restrict__ nlive, unsigned long long *cnt)
{
    const int n = nlive ? min(nmax, *nlive) : nmax;
    unsigned long long ni = 0, np = 0, ns = 0;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        const int w = items[i].w;
        ni += 1;
        np += (unsigned long long)(w & 255) * (unsigned long long)(w >> 8);
        ns += (unsigned long long)(w & 255) * MLP_PAIRS;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        ni += __shfl_xor(ni, o);
        np += __shfl_xor(np, o);
        ns += __shfl_xor(ns, o);
    }
    if ((threadIdx.x & 63) == 0 && ni) {
        atomicAdd(cnt, ni);
        atomicAdd(cnt + 1, np);
        atomicAdd(cnt + 2, ns);
    }
}

hipError_t launch_count_items(Workspace &ws, bool far, unsigned long long *cnt, hipStream_t st)
{
    const int4 *items = far ? ws.items_far.as<int4>() : ws.lazy ? ws.items_live.as<int4>() : ws.items.as<int4>();
    const int *nlive = far ? far_count(ws) : ws.lazy ? live_count(ws) : nullptr;
    const int nmax = far ? ws.n_items_far : ws.n_items;
    if (nmax <= 0 || !cnt) return hipSuccess;
    hipLaunchKernelGGL(k_count_items, dim3((unsigned)std::min((nmax + BLOCK - 1) / BLOCK, 256)), dim3(BLOCK), 0, st,
                       items, nmax, nlive, cnt);
    return hipGetLastError();
}

template <int R>
static void blend_launch(Workspace &ws, float *C, bool save, hipStream_t st, bool redo)
{
    // the second pass blends overflowed views again with every position's
    // radiance and adds the recorded far entries elsewhere
    const uint32_t mpos = redo ? 0xFFFFFFFFu : ws.mpos;
    const FarState fs{ws.frec.as<uint2>(), ws.fcnt.as<uint8_t>(), ws.ftile.as<uint8_t>(), ws.live.as<uint8_t>()};
    dim3 grid((unsigned)ws.n_chunks, (unsigned)ws.g.tiles);
    const uint32_t *tord = ws.tiles_ordered ? ws.torder.as<uint32_t>() : nullptr;
    if constexpr (R == 1) {
        grid.y = (unsigned)ws.g.tiles * 4;   // one workgroup per sub-tile
        const dim3 blk(BLEND1_THREADS);
        if (save)
            hipLaunchKernelGGL((k_blend_fwd1<true>), grid, blk, 0, st, ws.srec.as<float4>(),
                               ws.sbox.as<float4>(), ws.pval[ws.pairs_buf].as<uint32_t>(), ws.ranges.as<uint2>(), ws.rad.as<float2>(),
                               ws.d_chunks, ws.Kp, ws.g, C, ws.Tfin.as<float>(), ws.nlast.as<int>(),
                               ws.part.as<float>(), stat_words(ws), tord, ws.vflag.as<uint32_t>(), mpos, fs);
        else if (redo)
            hipLaunchKernelGGL((k_blend_fwd1<false, true>), grid, blk, 0, st, ws.srec.as<float4>(),
                               ws.sbox.as<float4>(), ws.pval[ws.pairs_buf].as<uint32_t>(), ws.ranges.as<uint2>(), ws.rad.as<float2>(),
                               ws.d_chunks, ws.Kp, ws.g, C, nullptr, nullptr, ws.part.as<float>(), nullptr, tord,
                               ws.vflag.as<uint32_t>(), mpos, fs);
        else
            hipLaunchKernelGGL((k_blend_fwd1<false>), grid, blk, 0, st, ws.srec.as<float4>(),
                               ws.sbox.as<float4>(), ws.pval[ws.pairs_buf].as<uint32_t>(), ws.ranges.as<uint2>(), ws.rad.as<float2>(),
                               ws.d_chunks, ws.Kp, ws.g, C, nullptr, nullptr, ws.part.as<float>(), nullptr, tord,
                               ws.vflag.as<uint32_t>(), mpos, fs);
    } else {
        if (save)
            hipLaunchKernelGGL((k_blend_fwd_multi<R, true>), grid, dim3(BLOCK), 0, st, ws.srec.as<float4>(),
                               ws.pval[ws.pairs_buf].as<uint32_t>(), ws.ranges.as<uint2>(), ws.rad.as<float2>(),
                               ws.d_chunks, ws.Kp, ws.g, C, ws.Tfin.as<float>(), ws.nlast.as<int>(),
                               ws.part.as<float>(), stat_words(ws), tord, ws.lazy ? ws.live.as<uint8_t>() : nullptr,
                               ws.vflag.as<uint32_t>(), mpos, fs);
        else if (redo)
            hipLaunchKernelGGL((k_blend_fwd_multi<R, false, false, true>), grid, dim3(BLOCK), 0, st,
                               ws.srec.as<float4>(), ws.pval[ws.pairs_buf].as<uint32_t>(), ws.ranges.as<uint2>(),
                               ws.rad.as<float2>(), ws.d_chunks, ws.Kp, ws.g, C, nullptr, nullptr,
                               ws.part.as<float>(), nullptr, tord, ws.lazy ? ws.live.as<uint8_t>() : nullptr,
                               ws.vflag.as<uint32_t>(), mpos, fs);
        else
            hipLaunchKernelGGL((k_blend_fwd_multi<R, false>), grid, dim3(BLOCK), 0, st, ws.srec.as<float4>(),
                               ws.pval[ws.pairs_buf].as<uint32_t>(), ws.ranges.as<uint2>(), ws.rad.as<float2>(),
                               ws.d_chunks, ws.Kp, ws.g, C, nullptr, nullptr, ws.part.as<float>(), nullptr, tord,
                               ws.lazy ? ws.live.as<uint8_t>() : nullptr, ws.vflag.as<uint32_t>(), mpos, fs);
    }
}

hipError_t launch_blend_fwd(Workspace &ws, float *C, bool save, hipStream_t st, bool redo)
{
    if (ws.n_chunks == 0) return hipSuccess;
    // grid y limit (one workgroup per sub-tile with one receiver per chunk)
    if ((int64_t)ws.g.tiles * (ws.R == 1 ? 4 : 1) > 65535) return hipErrorInvalidConfiguration;
    switch (ws.R) {
    case 1: blend_launch<1>(ws, C, save, st, redo); break;
    case 2: blend_launch<2>(ws, C, save, st, redo); break;
    case 4: blend_launch<4>(ws, C, save, st, redo); break;
    case 8: blend_launch<8>(ws, C, save, st, redo); break;
    default: blend_launch<16>(ws, C, save, st, redo); break;
    }
    return hipGetLastError();
}

// MLP work items of the positions past the prefix, for the views whose blend
// composited such a position (flags 4 and 8); one workgroup per view, any order
__global__ __launch_bounds__(BLOCK) void k_far_items(const int4 *__restrict__ vinfo, const uint32_t *__restrict__ vflag,
                                                     uint32_t mpos, const uint8_t *__restrict__ mark, int64_t Kp,
                                                     int4 *__restrict__ out, int *__restrict__ count)
{
    const int v = blockIdx.x;
    const uint32_t f = vflag[v];
    if (!(f & 12u)) return;
    const int4 vi = vinfo[v];   // (first receiver, receivers, visible, -)
    const int nb = (vi.z + MLP_PAIRS - 1) / MLP_PAIRS, nb0 = min(nb, (int)(mpos / MLP_PAIRS));
    const int nrg = (vi.y + MLP_RG - 1) / MLP_RG;
    if (!(f & 4u)) {
        // records only: the blocks they point into
        for (int sb = nb0 + threadIdx.x; sb < nb; sb += BLOCK) {
            if (!mark[((size_t)v * Kp) / MLP_PAIRS + sb]) continue;
            const int base = atomicAdd(count, nrg);
            const int s0 = sb * MLP_PAIRS;
            for (int a = 0; a < nrg; a++)
                out[base + a] = make_int4(v, s0, vi.x + a * MLP_RG,
                                          min(MLP_RG, vi.y - a * MLP_RG) | (min(MLP_PAIRS, vi.z - s0) << 8));
        }
        return;
    }
    // blended again: every block past the prefix
    const int n = (nb - nb0) * nrg;
    __shared__ int s_base;
    if (threadIdx.x == 0) s_base = n > 0 ? atomicAdd(count, n) : 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += BLOCK) {
        const int sb = nb0 + i / nrg, a = i - (i / nrg) * nrg;
        const int s0 = sb * MLP_PAIRS;
        out[s_base + i] = make_int4(v, s0, vi.x + a * MLP_RG,
                                    min(MLP_RG, vi.y - a * MLP_RG) | (min(MLP_PAIRS, vi.z - s0) << 8));
    }
}

// every view of a prefix render needs all its radiance (a radiance export):
// all blocks past the prefix, and the work-item count restarted
__global__ __launch_bounds__(BLOCK) void k_far_all(uint32_t *__restrict__ vflag, int V, int *__restrict__ count)
{
    for (int v = threadIdx.x; v < V; v += BLOCK) vflag[v] |= 4u;
    if (threadIdx.x == 0) *count = 0;
}

hipError_t launch_far_all(Workspace &ws, hipStream_t st)
{
    hipLaunchKernelGGL(k_far_all, dim3(1), dim3(BLOCK), 0, st, ws.vflag.as<uint32_t>(), ws.V, far_count(ws));
    return hipGetLastError();
}

int *far_count(Workspace &ws)
{
    return reinterpret_cast<int *>(emit_words(ws) + emit_word_count(ws.V, ws.Kp));
}

hipError_t launch_far_items(Workspace &ws, hipStream_t st)
{
    if (ws.V == 0) return hipSuccess;
    hipLaunchKernelGGL(k_far_items, dim3((unsigned)ws.V), dim3(BLOCK), 0, st, ws.d_vinfo, ws.vflag.as<uint32_t>(),
                       ws.mpos, ws.live.as<uint8_t>(), ws.Kp, ws.items_far.as<int4>(), far_count(ws));
    return hipGetLastError();
}


// Initial marks of the lazy path: blocks of views that take the weights pass
// start unmarked, those of the other views (few receivers: the pass would
// cost more than the MLP it saves) start marked; plus the live-item counter.
__global__ __launch_bounds__(BLOCK) void k_live_init(uint8_t *__restrict__ live, int64_t nblocks, int64_t bpv,
                                                     const int4 *__restrict__ vinfo, int *__restrict__ count)
{
    const int64_t b = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (b == 0) *count = 0;
    if (b >= nblocks) return;
    live[b] = vinfo[b / bpv].w ? 0 : 1;
}

// Compact the MLP work items whose position block is marked live (any order:
// items are independent) and count them.
__global__ __launch_bounds__(BLOCK) void k_live_items(const int4 *__restrict__ items, int nitems,
                                                      const uint8_t *__restrict__ live, int64_t Kp,
                                                      int4 *__restrict__ out, int *__restrict__ count)
{
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    bool lv = false;
    int4 it = make_int4(0, 0, 0, 0);
    if (i < nitems) {
        it = items[i];
        lv = live[((size_t)it.x * Kp + it.y) / MLP_PAIRS] != 0;
    }
    const uint64_t b = __ballot(lv);
    int base = 0;
    if ((threadIdx.x & 63) == 0 && b) base = atomicAdd(count, (int)__popcll(b));
    base = __shfl(base, 0);
    if (lv) out[base + count_below(b)] = it;
}

// Weights-only pass of the lazy TX path: marks the live position blocks of
// every view (one chunk per view with receivers, no outputs), then compacts
// the MLP work items of those blocks.
hipError_t launch_blend_weights(Workspace &ws, hipStream_t st)
{
    const int64_t nblocks = (int64_t)ws.V * ws.Kp / MLP_PAIRS;
    hipLaunchKernelGGL(k_live_init, dim3(nblk(nblocks)), dim3(BLOCK), 0, st, ws.live.as<uint8_t>(), nblocks,
                       ws.Kp / MLP_PAIRS, ws.d_vinfo, live_count(ws));
    if (ws.g.tiles > 65535) return hipErrorInvalidConfiguration;
    const uint32_t *tord = ws.tiles_ordered ? ws.torder.as<uint32_t>() : nullptr;
    if (ws.n_wchunks > 0)
        hipLaunchKernelGGL((k_blend_fwd_multi<1, false, true>), dim3((unsigned)ws.n_wchunks, (unsigned)ws.g.tiles),
                       dim3(BLOCK), 0, st, ws.srec.as<float4>(), ws.pval[ws.pairs_buf].as<uint32_t>(),
                       ws.ranges.as<uint2>(), ws.rad.as<float2>(), ws.d_wchunks, ws.Kp, ws.g, nullptr, nullptr,
                       nullptr, nullptr, nullptr, tord, ws.live.as<uint8_t>(), ws.vflag.as<uint32_t>(), 0xFFFFFFFFu,
                       FarState{nullptr, nullptr, nullptr, nullptr});
    if (ws.n_items > 0)
        hipLaunchKernelGGL(k_live_items, dim3(nblk(ws.n_items)), dim3(BLOCK), 0, st, ws.items.as<int4>(), ws.n_items,
                           ws.live.as<uint8_t>(), ws.Kp, ws.items_live.as<int4>(), live_count(ws));
    return hipGetLastError();
}

int *live_count(Workspace &ws)
{
    return reinterpret_cast<int *>(ws.live.as<char>() + live_count_offset(ws));
}

size_t live_count_offset(const Workspace &ws) { return ((size_t)ws.V * ws.Kp / MLP_PAIRS + 63) / 64 * 64; }

// output amplitude of every pixel, |C| = sqrt(Re^2 + Im^2 + eps) (App. E.2)
__global__ __launch_bounds__(BLOCK) void k_amplitude(const float *__restrict__ C, float *__restrict__ amp, int N,
                                                     size_t P)
{
    const size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= (size_t)N * P) return;
    const size_t j = i / P, p = i - j * P;
    const float re = C[2 * j * P + p], im = C[(2 * j + 1) * P + p];
    amp[i] = sqrtf(re * re + im * im + AMP_EPS);
}

hipError_t launch_amplitude(const float *C, float *amp, int N, size_t P, hipStream_t st)
{
    const size_t n = (size_t)N * P;
    if (n == 0 || !amp) return hipSuccess;
    hipLaunchKernelGGL(k_amplitude, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, C, amp, N, P);
    return hipGetLastError();
}

__global__ __launch_bounds__(BLOCK) void k_add_f32(float *__restrict__ out, const float *__restrict__ add, size_t n)
{
    const size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) out[i] += add[i];
}

hipError_t launch_add_f32(float *out, const float *add, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_f32, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, out, add, n);
    return hipGetLastError();
}

hipError_t launch_reduce_outputs(Workspace &ws, float *power, float *csum, hipStream_t st)
{
    if (ws.N == 0 || (!power && !csum)) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_out, dim3((unsigned)((ws.N + 3) / 4)), dim3(BLOCK), 0, st, ws.part.as<float>(), ws.N,
                       ws.g.tiles, ws.R == 1 ? 4 : 1, power, csum);
    return hipGetLastError();
}

}  // namespace rxgs
