// Stable segmented LSD radix sort of (u32 key, u32 value) pairs, one kernel
// per 8-bit digit ("onesweep" organisation).
//
// The keys are split into independent segments (one per view: the per-view
// depth sort, and the per-view padded pair lists).  One histogram kernel reads
// every key once and counts all digits of all passes per segment (or the
// caller has counted them while writing the keys).  Each pass is then a
// single kernel: the workgroup of index i takes tile i (4096 keys; segments
// are runs of whole tiles), ranks its keys stably, publishes its per-digit
// counts and obtains the counts of the earlier tiles of its segment by
// decoupled look-back, and writes its keys digit run by digit run.  Ranking is wave
// synchronous: each wave owns a contiguous quarter of the tile, takes its keys
// 64 at a time in index order, matches equal digits with 8 ballots and keeps
// running per-digit counts in LDS, so the only workgroup barriers are the ones
// around the look-back and the LDS staging of the tile.
//
// Keys equal to 0xFFFFFFFF (culled depth keys, padding of the pair lists) are
// dropped: the histogram does not count them and the first pass does not
// write them, so every segment's output is its surviving keys, in order, at
// the segment's start, and the later passes only touch that prefix (the
// segment's surviving count is the sum of its digit totals).
//
// Look-back progress: a workgroup only waits for tiles with a smaller index,
// whose workgroups were dispatched earlier; they publish their aggregates
// before waiting themselves, so every wait ends.  A wait is still bounded: on expiry the workgroup counts the digit totals of
// the segment's earlier tiles directly from their input keys (exact, slow),
// publishes them like a look-back result and adds one to the sort's
// fallback counter, so the order is right either way.
#include "device_common.h"

#include <cstdlib>

namespace rxgs {

namespace {

constexpr uint32_t LB_AGG = 1u << 30;    // status word: aggregate of this tile only
constexpr uint32_t LB_PRE = 1u << 31;    // status word: inclusive prefix up to this tile
constexpr uint32_t LB_MASK = LB_AGG - 1;
constexpr uint32_t SORT_DROP = 0xFFFFFFFFu;   // dropped key

struct SortSeg {
    uint32_t seg_blocks;   // uniform segments of this many tiles (0: table or one segment)
    const int4 *tab;       // per 4096-key unit: (first unit of its segment, units, segment id, 0)
    uint32_t scale;        // tiles per 4096-key unit
};

__device__ __forceinline__ void tile_segment(uint32_t tile, const SortSeg &sm, uint32_t &seg, uint32_t &first)
{
    if (sm.tab) {
        const int4 e = sm.tab[tile / sm.scale];
        first = (uint32_t)e.x * sm.scale;
        seg = (uint32_t)e.z;
    } else if (sm.seg_blocks) {
        seg = tile / sm.seg_blocks;
        first = seg * sm.seg_blocks;
    } else {
        seg = 0;
        first = 0;
    }
}

// digit counts of every pass, per segment: hist[seg][pass][256]
template <int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_sort_hist(const uint32_t *__restrict__ keys, uint32_t n, int passes,
                                                     SortSeg sm, uint32_t *__restrict__ hist)
{
    constexpr int TILEN = BLOCK * ITEMS;
    __shared__ uint32_t h[4][4][256];   // [pass][wave][digit]
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
        for (int ww = 0; ww < 4; ww++) h[p][ww][t] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * TILEN;
    uint32_t k[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const size_t idx = base + (size_t)i * BLOCK + t;
        k[i] = idx < n ? keys[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        if (base + (size_t)i * BLOCK + t < n && k[i] != SORT_DROP)
            for (int p = 0; p < passes; p++) atomicAdd(&h[p][w][(k[i] >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    uint32_t seg, first;
    tile_segment(blockIdx.x, sm, seg, first);
    for (int p = 0; p < passes; p++) {
        const uint32_t c = h[p][0][t] + h[p][1][t] + h[p][2][t] + h[p][3][t];
        if (c) atomicAdd(&hist[((size_t)seg * passes + p) * 256 + t], c);
    }
}

template <int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_sort_pass(const uint32_t *__restrict__ kin,
                                                     const uint32_t *__restrict__ vin,
                                                     uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                     uint32_t n, int pass, int passes, SortSeg sm, int flags,
                                                     const uint32_t *__restrict__ hist, uint32_t *status,
                                                     uint32_t *seg_kept, uint32_t *err, int spin_max)
{
    constexpr int TILEN = BLOCK * ITEMS;
    constexpr int WCH = 64 * ITEMS;   // keys per wave
    __shared__ uint32_t s_key[TILEN];
    __shared__ uint32_t s_val[TILEN];
    __shared__ uint32_t s_wc[4][256];   // per-wave running digit counts, then per-wave digit starts
    __shared__ uint32_t s_loc[256];     // tile-local start of each digit
    __shared__ uint32_t s_glob[256];    // output start of each digit for this tile
    __shared__ uint32_t s_w[4];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int shift = 8 * pass;
    // the workgroup's tile is its index, and its segment follows from it
    // (segments are runs of whole tiles); workgroups are dispatched in index
    // order, so a look-back waits only for tiles already dispatched (and the
    // wait is bounded in any case)
    const uint32_t tile = blockIdx.x;
    uint32_t seg, first;
    tile_segment(tile, sm, seg, first);
    const size_t tile0 = (size_t)tile * TILEN, seg0 = (size_t)first * TILEN;
    const size_t base = tile0 + (size_t)w * WCH;
    // the tile's keys, loaded first so that their latency overlaps the scan
    // of the segment's digit totals (positions past the segment's surviving
    // prefix are dropped below)
    const size_t lim0 = min((size_t)n, tile0 + TILEN);
    uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
        const size_t idx = base + (size_t)r * 64 + lane;
        const bool in = idx < lim0;
        key[r] = in ? kin[idx] : SORT_DROP;
        // (first pass with SORT_VALS_INDEX: a key's value is its index in its segment)
        val[r] = !in ? 0u : (pass == 0 && (flags & SORT_VALS_INDEX)) ? (uint32_t)(idx - seg0) : vin[idx];
    }
#pragma unroll
    for (int ww = 0; ww < 4; ww++) s_wc[ww][t] = 0;
    // digit starts in the segment (from its digit totals) and its surviving count
    uint32_t seg_n;
    const uint32_t dbase = block_exclusive_scan(hist[((size_t)seg * passes + pass) * 256 + t], seg_n, s_w);
    if (pass == 0 && seg_kept && tile == first && t == 0) seg_kept[(size_t)seg * KEPT_STRIDE] = seg_n;
    // input positions of this tile that hold keys: all (first pass), or the
    // part of the segment's surviving prefix inside the tile (later passes)
    size_t lim = lim0;
    if (pass > 0) {
        lim = min(lim, seg0 + seg_n);
        if (tile0 >= lim) return;   // uniform; later tiles of the segment are empty too
#pragma unroll
        for (int r = 0; r < ITEMS; r++)
            if (base + (size_t)r * 64 + lane >= lim) key[r] = SORT_DROP;
    }
    // stable rank inside the wave's chunk: the keys of one round are matched by
    // digit; a digit's running count is read by all its lanes, then advanced by
    // its lowest lane (LDS operations of one wave execute in program order)
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
        const bool valid = key[r] != SORT_DROP;
        const uint32_t d = (key[r] >> shift) & 255u;
        const uint64_t m = match_key8(d, __ballot(valid));
        const uint32_t below = (uint32_t)count_below(m);
        const uint32_t before = s_wc[w][d];
        rank[r] = before + below;
        if (valid && below == 0) s_wc[w][d] = before + (uint32_t)__popcll(m);
    }
    __syncthreads();
    const uint32_t c0 = s_wc[0][t], c1 = s_wc[1][t], c2 = s_wc[2][t], c3 = s_wc[3][t];
    const uint32_t cnt = c0 + c1 + c2 + c3;

    // decoupled look-back over the earlier tiles of this segment, digit t
    uint32_t *mine = status + (size_t)tile * 256 + t;
    uint32_t excl = 0;
    bool gave_up = false;
    if (tile == first) {
        __hip_atomic_store(mine, LB_PRE | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(mine, LB_AGG | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // eight predecessors in flight per step; tiles before the segment's
        // first count as an empty prefix (spin_max < 0: no look-back at all)
        int64_t j = (int64_t)tile - 1;
        int spins = 0;
        while (spin_max >= 0) {
            uint32_t w8[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int64_t idx = j - q;
                w8[q] = idx >= (int64_t)first ? __hip_atomic_load(status + (size_t)idx * 256 + t, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT)
                                              : LB_PRE;
            }
            int q = 0;
            bool done = false;
            for (; q < 8; q++) {
                if (w8[q] == 0) break;
                excl += w8[q] & LB_MASK;
                if (w8[q] & LB_PRE) {
                    done = true;
                    break;
                }
            }
            if (done) break;
            j -= q;
            if (q < 8) {   // predecessor j has not published yet
                if (++spins > spin_max) {
                    gave_up = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        gave_up |= spin_max < 0;
        if (!gave_up)
            __hip_atomic_store(mine, LB_PRE | (excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // an expired wait: the digit totals of the segment's earlier tiles, counted
    // from their input keys (positions seg0 .. tile0 hold keys in every pass)
    if (__syncthreads_or(gave_up)) {
        s_glob[t] = 0;
        __syncthreads();
        const size_t e0 = (size_t)first * TILEN, e1 = (size_t)tile * TILEN;
        for (size_t i = e0 + t; i < e1; i += BLOCK) {
            const uint32_t k = kin[i];
            if (k != SORT_DROP) atomicAdd(&s_glob[(k >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (gave_up) {
            excl = s_glob[t];
            __hip_atomic_store(mine, LB_PRE | (excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (t == 0) atomicAdd(err, 1u);
        __syncthreads();
    }

    // digit starts in the tile
    uint32_t tile_kept;
    const uint32_t loc = block_exclusive_scan(cnt, tile_kept, s_w);
    s_glob[t] = first * (uint32_t)TILEN + dbase + excl;
    s_loc[t] = loc;
    s_wc[0][t] = loc;
    s_wc[1][t] = loc + c0;
    s_wc[2][t] = loc + c0 + c1;
    s_wc[3][t] = loc + c0 + c1 + c2;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
        if (key[r] != SORT_DROP) {
            const uint32_t pos = s_wc[w][(key[r] >> shift) & 255u] + rank[r];
            s_key[pos] = key[r];
            s_val[pos] = val[r];
        }
    }
    __syncthreads();
    // write out digit run by digit run: consecutive slots go to consecutive addresses
    for (uint32_t i = t; i < tile_kept; i += BLOCK) {
        const uint32_t k = s_key[i];
        const uint32_t d = (k >> shift) & 255u;
        const uint32_t o = s_glob[d] + (i - s_loc[d]);
        if (o < n) {
            if (pass + 1 < passes || !(flags & SORT_VALS_ONLY)) kout[o] = k;
            vout[o] = s_val[i];
        }
    }
}

// Bound of a look-back wait, in polls of a predecessor's status.
// RXGS_SORT_SPIN_LIMIT overrides it (a negative value skips the look-back and
// takes the direct count in every tile after a segment's first: the path an
// expired wait takes, forced from the host so that it can be tested).
int sort_spin_limit()
{
    const char *e = std::getenv("RXGS_SORT_SPIN_LIMIT");
    if (e && e[0]) return std::atoi(e);
    return 1 << 20;
}

template <int ITEMS>
hipError_t sort_run(DevBuf *keys, DevBuf *vals, DevBuf &wsb, int &cur, uint32_t n, int bits, int nseg,
                    int64_t seg_len, const int4 *segtab, bool zeroed, bool counted, uint32_t *seg_kept,
                    int flags, hipStream_t st)
{
    constexpr uint32_t TILEN = BLOCK * ITEMS;
    const uint32_t ntiles = (n + TILEN - 1) / TILEN;
    const int passes = (bits + 7) / 8;
    SortSeg sm;
    sm.seg_blocks = seg_len > 0 ? (uint32_t)(seg_len / TILEN) : 0u;
    sm.tab = segtab;
    sm.scale = SORT_TILE / TILEN;
    const size_t words = sort_ws_bytes(n, bits, nseg) / 4;
    if (wsb.cap < words * 4) return hipErrorOutOfMemory;
    uint32_t *hist = wsb.as<uint32_t>();
    uint32_t *status = hist + (size_t)nseg * passes * 256;
    uint32_t *err = status + (size_t)passes * ntiles * 256;
    if (!zeroed) {
        hipError_t e = launch_fill_u32(hist, 0u, words, st);
        if (e != hipSuccess) return e;
    }
    if (!counted)
        hipLaunchKernelGGL(k_sort_hist<ITEMS>, dim3(ntiles), dim3(BLOCK), 0, st, keys[cur].as<uint32_t>(), n, passes,
                           sm, hist);
    const int spin_max = sort_spin_limit();
    for (int p = 0; p < passes; p++) {
        hipLaunchKernelGGL(k_sort_pass<ITEMS>, dim3(ntiles), dim3(BLOCK), 0, st, keys[cur].as<uint32_t>(),
                           vals[cur].as<uint32_t>(), keys[cur ^ 1].as<uint32_t>(), vals[cur ^ 1].as<uint32_t>(), n, p,
                           passes, sm, flags, hist, status + (size_t)p * ntiles * 256, seg_kept, err, spin_max);
        cur ^= 1;
    }
    return hipGetLastError();
}

}  // namespace

int sort_items_for(uint32_t n) { return n <= SMALL_SORT ? 4 : 16; }

uint32_t *sort_fallback_word(DevBuf &wsb, uint32_t n, int bits, int nseg)
{
    if (n == 0 || bits <= 0 || nseg <= 0 || !wsb.p) return nullptr;
    const uint32_t tilen = BLOCK * (uint32_t)sort_items_for(n);
    const size_t ntiles = (n + tilen - 1) / tilen;
    const size_t passes = (size_t)(bits + 7) / 8;
    return wsb.as<uint32_t>() + (size_t)nseg * passes * 256 + passes * ntiles * 256;
}

size_t sort_ws_bytes(uint32_t n, int bits, int nseg)
{
    const uint32_t tilen = BLOCK * (uint32_t)sort_items_for(n);
    const size_t ntiles = (n + tilen - 1) / tilen;
    const size_t passes = (size_t)(std::max(bits, 1) + 7) / 8;
    return ((size_t)std::max(nseg, 1) * passes * 256 + passes * ntiles * 256 + 64) * 4;
}

hipError_t sort_pairs_u32(DevBuf *keys, DevBuf *vals, DevBuf &wsb, int &cur, uint32_t n, int bits, int nseg,
                          int64_t seg_len, const int4 *segtab, hipStream_t st, bool zeroed, bool counted,
                          uint32_t *seg_kept, int flags)
{
    if (n == 0 || bits <= 0) return hipSuccess;
    if (bits > 32 || nseg <= 0 || (counted && !zeroed)) return hipErrorInvalidValue;
    if (sort_items_for(n) == 4)
        return sort_run<4>(keys, vals, wsb, cur, n, bits, nseg, seg_len, segtab, zeroed, counted, seg_kept, flags,
                           st);
    return sort_run<16>(keys, vals, wsb, cur, n, bits, nseg, seg_len, segtab, zeroed, counted, seg_kept, flags, st);
}

}  // namespace rxgs
