// Internal declarations of librxgs (MI355X / gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "rxgs.h"

namespace rxgs {

constexpr int TILE = RXGS_TILE;          // 16 x 16 pixel tiles, one pixel per thread
constexpr int BLOCK = 256;               // threads per workgroup (4 wave64)
constexpr int SORT_ITEMS = 16;           // keys per thread in the radix sort
constexpr int SORT_TILE = BLOCK * SORT_ITEMS;  // 4096 keys per sort block
constexpr int FEAT = RXGS_FEAT_DIM;
constexpr int ENC = 36;
constexpr int HID = 64;
constexpr int MLP_IN = ENC + FEAT;
constexpr int MLP_RG = 16;               // receivers per MLP work item
constexpr int MLP_PAIRS = 32;            // sorted positions per MLP work item
constexpr int LAZY_MIN_RX = 4;           // receivers of a TX view for its weights-only pass
constexpr int64_t NEAR_LIMIT = 4096;     // nearest depth-sorted entries emitted per view first
constexpr uint32_t PREFIX_POS = 4096;    // sorted positions whose radiance the first blend pass gets (TX)
constexpr uint32_t PREFIX_POS_RX = 8192; // the same for RX views (a view is one receiver)
constexpr int FAR_RECORDS = 16;          // recorded far entries per pixel (FarState)
constexpr int AMAX_SLOTS = 128;          // activation-bound words after the view counters
constexpr int STAT_SLOTS = 64;           // u64 slots per render statistic (spread atomics)
constexpr int STAT_WORDS = 4 * STAT_SLOTS;   // four statistics, u64 each
constexpr uint32_t SMALL_SORT = 1u << 20;  // sorts up to this length use 1024-key blocks
constexpr int EM2_PER = 1;               // pair emission: 256-entry sub-chunks per workgroup
constexpr int EM2_CHUNK = BLOCK * EM2_PER;
constexpr int BIN_MAX_TILES = 255;       // grids up to this many tiles place their pairs without a pair sort
constexpr int BIN_DIFF_WORDS = 512;      // LDS words of the per-tile difference counts (tiles_y x (tiles_x + 1))
constexpr int KEPT_STRIDE = 32;          // words between the per-view kept counts the depth sort leaves
constexpr int SORT_VALS_INDEX = 1;       // sort flag: a key's value is its index in its segment (not read)
constexpr int SORT_VALS_ONLY = 2;        // sort flag: the sorted keys are not needed (last pass writes values only)
constexpr int BIN_WIN = 2048;            // pair slots per placement unit of the direct binning
constexpr int BIN_CHUNK_MAX = 1024;      // most entries of a chunk of the first emission
constexpr int BIN_GROUP = 2;             // placement units of one chunk per workgroup (renders with many chunks)

// Method constants (Alg. 1 compositing and the readings of its unstated values).
constexpr float ALPHA_MIN = 1.0f / 255.0f;   // skip threshold on the blend weight
constexpr float W_MAX = 0.99f;               // blend weight clamp
// log2 o at or above which an entry's blend weight may reach the clamp: its
// exponent peaks at log2 o, and this sits 0.035 below log2 0.99 (= -0.0145),
// far above the FP32 error of the exponent
constexpr float LOG2_W_MAX = -0.05f;
constexpr float T_EPS = 1e-4f;               // early-termination transmittance
constexpr double DILATE = 0.3;               // px^2 added to the projected covariance
constexpr float NEAR2 = 0.04f;               // cull Gaussians closer than 0.2 m
constexpr double H_MIN = 1e-6;               // horizontal distance floor (poles)
constexpr double PAD_REL = 1e-4;             // conservative padding of the
constexpr double PAD_ABS = 0.01;             //   binning ellipse box, px
constexpr float AMP_EPS = 1e-8f;             // amplitude stabiliser, sqrt(Re^2 + Im^2 + eps)

struct DevGrid {
    int H, W, tiles_x, tiles_y, tiles;
    double el0, del, daz, idel, idaz;
};

// Where a context's device buffers come from: the caller's allocator
// callbacks when given, else hipMalloc / hipFree; or a fixed region whose
// buffers are carved in order and never freed one by one (the
// allocation-free entry point: the region is rewound before each call).
struct Allocator {
    rxgs_alloc_fn alloc = nullptr;
    rxgs_free_fn free = nullptr;
    void *user = nullptr;
    int device = 0;
    char *base = nullptr;   // fixed region (nullptr: none)
    size_t cap = 0, used = 0;
};

// grow-only device buffer
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    Allocator *al = nullptr;   // its source (nullptr: hipMalloc)
    template <class T> T *as() const { return static_cast<T *>(p); }
};

struct Scene {
    int64_t K = 0;
    bool has_features = false;
    bool geometry_only = false;   // no radiance of its own (conditioning model only)
    bool valid = false;
    uint64_t version = 0;
    DevBuf soa;    // 11 x K: x, y, z, ls0, ls1, ls2, qw, qx, qy, qz, logit
    DevBuf rad;    // K x 2
    DevBuf feat;   // K x 32
    float fmax = 0.f;   // largest |feature|
};

struct Mlp {
    bool valid = false;
    uint64_t version = 0;
    DevBuf raw;    // RXGS_MLP_NPARAM
    DevBuf w2a;    // [2][32][64]  W2[32 mb + l % 32][hid_of(l / 32, t)]
    DevBuf w2b;    // [2][32][64]  W2[hid_of(l / 32, t)][32 ib + l % 32]
    DevBuf tab;    // [2 h][2 mb][16 r] float4 (W3[0][d], W3[1][d], b2[d], 0)
    // split-FP16 forward: W2 * 2^wexp as FP16 (hi, lo) pairs in the MFMA
    // 32x32x16 A-operand layout, [2 part][2 mb][4 q][64 lane] x 8 halves,
    // element i = W2[32 mb + lane % 32][hid_of(lane / 32, 8 q + i)]
    DevBuf w2h;
    DevBuf tabh;   // as tab, with (W3 * 2^-wexp, b2 * 2^wexp)
    int wexp = 0;
    // the Gaussians' layer-1 term inside the pair kernel: W1[:, 36:] * 2^w1exp
    // split to FP16 (hi, lo) in the A-operand layout, [2 part][2 mb][2 q][64]
    // x 8 halves; b1 * 2^w1exp per lane half in accumulator order; per-row
    // sums of |W1[:, 36:]| and |b1| for the activation bound
    DevBuf w1h;
    DevBuf b1tab;
    int w1exp = 0;
    bool w1_ok = false;
    double w1abs[64] = {};
    double b1abs[64] = {};
    bool fp32 = false;   // layer 2 on FP32 MFMA instead: RXGS_MLP_FP32=1, or the
                         // rescaled tables would not be exact
};

// The receiver-conditioned radiance model (rxgs_rxcond_upload).  Component
// tables are stored in the basis walk's order (rxcond.hip: lane half h walks
// the orders |m| of parity h, m ascending, degree ascending, +m before -m).
// Offsets (floats) of the parts of the flat conditioning parameters.
struct RcOffsets {
    size_t w, e, g1, gb1, g2, gb2, g3, gb3, l1, lb1, l2, lb2, l3, lb3, total;
};
RcOffsets rc_offsets(int L, int C, int F);

struct RxCond {
    bool valid = false;
    uint64_t version = 0;
    uint64_t scene_version = 0;
    int kind = 0, lmax = 0, L = 0, C = 1, F = 1, S = 16, G = 128;
    int n0 = 0;                 // walk positions of lane half 0 (half 1 follows)
    RcOffsets off{};
    DevBuf coef;                // K x L x C float2, walk order
    DevBuf params;              // the flat parameters as uploaded
    DevBuf comp;                // L x 64: b1 + W1 [deg/m, ord/m; e_l] per component, walk order
    DevBuf walk;                // L int: component index deg^2 + deg + ord at each walk position
    DevBuf ctab;                // 13 x 13 float4 (N_lm, (2l-1)/(l-m), (l+m-1)/(l-m), 0)
    DevBuf tprobe;              // S f64 probe fractions t_s
    DevBuf occ;                 // G^3 occupancy
    DevBuf w2t;                 // local W2 in the FP32 MFMA A-operand layout [2 blk][32 t][64 lane]
    double lo[3] = {}, hi[3] = {}, inv[3] = {}, vs[3] = {};   // grid box, G / (hi - lo), (hi - lo) / G
};

// radiance of a render: the scene's own (direct or conditioning MLP) or a
// conditioning model's
enum { RSRC_SCENE = 0, RSRC_RXCOND = 1 };

struct Workspace {
    Allocator *al = nullptr;   // source of its device buffers (nullptr: the context's)
    int rsrc = RSRC_SCENE;     // radiance source of the last render
    int Nrx = 0, Ch = 1;       // receivers and channels (rows N = Nrx x Ch)
    int rx_max = 1;            // most receivers of one view
    bool use_items = false;    // radiance evaluated per MLP work item (MLP or conditioning model)
    uint64_t rxc_version = 0;
    DevBuf rgam;               // Nrx x 64 receiver term of the conditioning's global layer 1
    DevBuf rab;                // Nrx x L x C float4 global modulation (1 + alpha, beta), walk order
    DevBuf rloc;               // Nrx x Kp x C float4 local modulation (1 + alpha', beta') per sorted position
    bool fixed_host = false;   // h_pinned is a fixed buffer made at set-up (never regrown)
    size_t req_bytes = 0;      // device bytes the last render's buffers asked for
    // deterministic backward (rxgs_set_deterministic): the forward kept every
    // position's radiance and the emission order of the pairs
    bool det = false;
    DevBuf gP;                 // [block of a view][Dpad][8] record-gradient partials per pair slot
    DevBuf dSP;                // [row of a view][Dpad][2] dL/ds partials per pair slot
    DevBuf oinv;               // V x K int: sorted position of each (view, Gaussian), -1 if not visible
    DevBuf rank;               // V x Kp / 32 int: slot of each marked position block, -1 unmarked
    DevBuf lcnt;               // per 1024 blocks: marked-block offsets, then their total
    DevBuf dLv;                // [slot][receiver group][32][64] Gaussian terms of the MLP backward
    DevBuf dGp;                // [slot][row of the view][64] receiver terms of the MLP backward
    // sizes of the last render
    int mode = 0, V = 0, N = 0, Q = 0, R = 1;
    int64_t K = 0, Kp = 0, D = 0, Dpad = 0, nvis_total = 0;
    uint64_t scene_version = 0, mlp_version = 0;
    bool valid = false;
    bool use_mlp = false;
    DevGrid g{};
    std::vector<int> h_nvis;          // V
    std::vector<int> h_rxview;        // N
    int n_chunks = 0, n_items = 0, n_tslots = 0;

    DevBuf centres;   // V x 3
    DevBuf rxpos;     // N x 3
    DevBuf ext;       // V x Kp float4 (u, v, rup, rvp), saved states only
    DevBuf rawkey;    // V x Kp u32, saved states only
    DevBuf opac;      // V x Kp f32, saved states only
    DevBuf skey[2];   // V x Kp u32 sort keys (ping-pong)
    DevBuf sval[2];   // V x Kp u32 sort values
    int sorted_buf = 0;
    DevBuf ggeo;      // K x 48 B view-independent projection terms of every Gaussian
    DevBuf qcull;     // K f32 elevation-cull bound of every Gaussian
    DevBuf srec;      // V x Kp x 2 float4 blend records of the visible entries in depth order
    DevBuf sbox;      // V x Kp float4 binning boxes (u, v, rup, rvp), same order
    DevBuf vorder;    // V x Kp u32 Gaussian of each visible entry, same order
    DevBuf poff;      // V x Kp u32 first pair slot of each visible entry within its view
    DevBuf desc;      // small descriptors copied from the host in one transfer:
    int *d_rxview = nullptr;       //   N: view of each receiver
    int4 *d_chunks = nullptr;      //   blend chunks (view, first receiver, receivers, T slot)
    int4 *d_vinfo = nullptr;       //   V: (first receiver, receivers, visible Gaussians, 0)
    uint32_t *d_item_off = nullptr;  // V + 1: first MLP work item of each view
    uint32_t *d_chunk_off = nullptr;  // V + 1: first pair-emission chunk (EM2_CHUNK visible entries) of each view
    int n_emit_chunks = 0;
    uint32_t *d_pbase = nullptr;   //   V: start of each view's segment of the pair arrays
    uint32_t *d_pcount = nullptr;  //   V: pairs of each view
    int4 *d_segtab = nullptr;      //   per 4096 pair slots: (first unit, units, view, 0) of its segment
    const float *centres_p = nullptr;  // view centres (the caller's or the saved copy)
    const float *rxpos_p = nullptr;    // receiver positions (the caller's or the saved copy)
    std::vector<uint32_t> h_pbase;    // V
    std::vector<uint32_t> h_pcount;   // V: pairs of each view
    DevBuf pkey[2];   // Dpad u32: local tile id, 0xFFFFFFFF for padding
    DevBuf pval[2];   // D u32
    int pairs_buf = 0;
    DevBuf ranges;    // V x tiles uint2
    DevBuf torder;    // V x tiles u32: tiles by list length, longest first
    bool tiles_ordered = false;
    bool items_built = false;   // the MLP work items were expanded with the ranges
    DevBuf rad;       // N x Kp float2
    DevBuf Lp;        // K x 64
    DevBuf Gp;        // N x 64
    DevBuf items;     // MLP work items (view, s0, first receiver, receivers | valid positions << 8)
    DevBuf Tfin;      // S x H x W
    DevBuf nlast;     // S x H x W
    DevBuf part;      // N x tiles x 3
    DevBuf counters;  // u64 per view: [2 v] visible Gaussians, [2 v + 1] pairs; then the
                      // activation bounds, render statistics and the emission's look-back words
    DevBuf hist;      // radix sort scratch (depth sort)
    DevBuf hist_b;    // radix sort scratch (pair sort); per-view tile counts at its start
    // direct binning (at most BIN_MAX_TILES tiles): per chunk of the first
    // emission its pairs per tile (then its start in each tile's list), per
    // chunk (first visible entry, visible entries), per view its list
    // lengths and its live chunks
    DevBuf bins;
    bool direct_bins = false;
    int em_cpv = 0, em_chunk = 0;   // chunks of the first emission per view, kept entries per chunk
    int bin_group = 1;              // placement units per workgroup of the direct binning
    bool live_cleared = false;      // the ranges launch cleared the prefix path's position-block marks
    DevBuf nvis_d;    // V int
    // backward scratch
    DevBuf dS;        // N x Kp float2
    DevBuf g2d;       // V x Kp x 8 (u, v, a, b, c, o partials)
    DevBuf dL;        // K x 64
    DevBuf dG;        // N x 64
    DevBuf mpart;     // per-wave partial sums of the MLP backward
    DevBuf w1part;    // per-chunk partial sums of dW1 (Gaussian part)
    DevBuf mred;      // FP64 group sums of the two-stage column reductions
    DevBuf gfeat_tmp; // K x 32 feature gradients before they are added (accumulating backward)
    DevBuf gmlp_tmp;  // MLP gradients before they are added (accumulating backward)
    DevBuf live;      // per (view, 32 sorted positions): composited (lazy forward) or some dL/ds nonzero (backward)
    DevBuf pterm;     // K x PROJ_TERM_BYTES: per-Gaussian terms of the projection backward
    DevBuf pacc;      // K x PACC_STRIDE floats: per-Gaussian sums of the projection backward
    DevBuf items_live;   // MLP work items of the live blocks (lazy forward)
    bool lazy = false;   // this render evaluates the pair MLP on live blocks only
    uint32_t limit = 0xFFFFFFFFu;   // depth-sorted entries emitted per view (the nearest)
    uint32_t mpos = 0xFFFFFFFFu;    // pair MLP first on sorted positions below this (prefix radiance)
    int R_max = 1;       // most receivers of one view
    DevBuf items_far;    // MLP work items past the prefix of the views that need them
    DevBuf frec, fcnt, ftile;   // composited entries past the prefix: records, counts, tile marks
    int n_items_far = 0; // their largest possible number
    bool rad_complete = true;   // every visible position's radiance is evaluated
    bool exports_ready = false; // binning boxes, raw keys and opacities computed (saved states, on export)
    DevBuf vflag;        // per view bits: 1 entries cut, 2 a pixel open after a cut, 4 composited past the prefix
    int n_wchunks = 0;   // weights-pass chunks: one per view with receivers
    int4 *d_wchunks = nullptr;
    // host staging (pinned) and the events guarding it
    void *h_pinned = nullptr;
    size_t h_pinned_cap = 0;
    hipEvent_t staged = nullptr;   // last host-to-device copy out of h_pinned
    hipEvent_t counted = nullptr;  // counters copied to h_pinned
    hipEvent_t done = nullptr;     // end of the last render or backward into this workspace
    int pair_bits = 0;             // key bits of the last pair sort
};

// Per-stage event timing (rxgs_profile_enable / rxgs_profile_read).
struct Profiler {
    bool on = false;
    struct Pending {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::vector<std::string> names;
    std::vector<int64_t> launches;
    std::vector<double> ms;
    unsigned long long *dcount = nullptr;   // device: MLP work items, pairs, slots of profiled renders
    int stage_id(const char *name);
    hipEvent_t take();
    void flush();
    void release_all();
};

// Records an event pair around one stage when profiling is on.
struct StageMark {
    Profiler *p;
    int stage = -1;
    hipEvent_t a = nullptr;
    hipStream_t st;
    StageMark(Profiler &prof, const char *name, hipStream_t s);
    ~StageMark();
};

}  // namespace rxgs

struct rxgs_ctx {
    int device = 0;
    rxgs::DevGrid g{};
    rxgs_grid grid{};
    rxgs::Scene scene;
    rxgs::Mlp mlp;
    rxgs::RxCond rxc;       // conditioning model of the paper's radiance path
    rxgs::Workspace ws;     // used when the caller passes no saved state
    rxgs::DevBuf stage;     // scene upload staging
    std::string err;
    uint64_t version_counter = 0;
    std::vector<rxgs_saved *> saved;   // live saved states
    rxgs::Profiler prof;
    bool near_cut = false;     // emit each view's nearest entries first (rxgs_set_near_cut)
    bool deterministic = false;   // saved renders and their backward sum in fixed orders (rxgs_set_deterministic)
    bool pair_sort = false;       // bin through the pair sort on every grid (RXGS_PAIR_SORT=1), not only large ones
    int64_t views_redone = 0;  // views redone over all their entries
    hipStream_t aux = nullptr; // private non-blocking stream of the saved-state queries and exports
    rxgs::Allocator alloc;     // the context's device allocations
    rxgs::Allocator fixed;     // this device's copy of the static scratch array (rxgs_render_noalloc)
    rxgs_saved *noalloc = nullptr;   // the allocation-free entry point's workspace, carved from `fixed`
};

struct rxgs_saved {
    rxgs_ctx *ctx = nullptr;
    rxgs::Workspace ws;
    // false: the object is only a private workspace (a serving slot): renders
    // into it keep no state for the backward or the exports
    bool keep = true;
};

namespace rxgs {

// ---- launch wrappers (kernels.hip) ----
// view-independent projection terms (which also clear the counters and the
// depth sort's scratch), then the depth keys and the sort's digit totals
hipError_t launch_project(const Scene &sc, const float *centres, int V, int64_t Kp, const DevGrid &g,
                          Workspace &ws, size_t counter_words, size_t sort_words, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t st);
// a saved state's binning boxes, raw keys and opacities, from its own centres
hipError_t launch_project_exports(Workspace &ws, hipStream_t st);
// zeroes several buffers (u32 words) in one launch (backward.hip)
constexpr int ZERO_RANGES = 12;
struct ZeroRanges {
    uint32_t *p[ZERO_RANGES];
    size_t len[ZERO_RANGES];
    int n = 0;
    void add(void *ptr, size_t words)
    {
        if (ptr && words) {
            p[n] = static_cast<uint32_t *>(ptr);
            len[n++] = words;
        }
    }
};
hipError_t launch_zero_ranges(const ZeroRanges &z, hipStream_t st);
// zeroes the visible positions' words of per-view (segview NULL) or
// per-receiver (segview: receiver -> view) rows of Kp x wpr words (backward.hip)
hipError_t launch_zero_visible(uint32_t *p, int64_t Kp, int wpr, const unsigned long long *counters,
                               const int *segview, int nseg, hipStream_t st);
// sort.hip: stable segmented radix sort of (key, value) pairs by the low
// `bits` key bits; segments of seg_len keys (a multiple of 4096), or given per
// 4096-key unit by segtab; wsb holds sort_ws_bytes(n, bits, nseg) bytes and
// keeps the per-segment digit totals at its start; zeroed: the caller has
// cleared those bytes already on this stream; counted: the caller has also
// added every key's digits to those totals (the histogram pass is skipped);
// seg_kept: the first pass writes each segment's surviving key count there
// (KEPT_STRIDE words apart)
hipError_t sort_pairs_u32(DevBuf *keys, DevBuf *vals, DevBuf &wsb, int &cur, uint32_t n, int bits, int nseg,
                          int64_t seg_len, const int4 *segtab, hipStream_t st, bool zeroed = false,
                          bool counted = false, uint32_t *seg_kept = nullptr, int flags = 0);
size_t sort_ws_bytes(uint32_t n, int bits, int nseg);
// the sort's counter of look-back waits that expired and took the direct count
// (inside wsb; zeroed with the rest of the scratch)
uint32_t *sort_fallback_word(DevBuf &wsb, uint32_t n, int bits, int nseg);
hipError_t launch_emit1(const Scene &sc, Workspace &ws, const DevGrid &g, hipStream_t st);
hipError_t launch_emit2(Workspace &ws, const DevGrid &g, size_t sort_words, hipStream_t st);
// direct binning: the first emission's chunking (sets em_cpv, em_chunk), the
// bytes of the bins buffer, the per-view scan and the placement of the pairs
void emit1_chunking(Workspace &ws);
size_t bins_bytes(int V, int cpv);
hipError_t launch_bin_scan(Workspace &ws, const DevGrid &g, hipStream_t st);
hipError_t launch_bin_pairs(Workspace &ws, const DevGrid &g, hipStream_t st);
uint32_t *emit_words(Workspace &ws);
size_t emit_word_count(int V, int64_t Kp);
hipError_t launch_ranges(Workspace &ws, const DevGrid &g, hipStream_t st);
hipError_t launch_rad_direct(const Scene &sc, Workspace &ws, hipStream_t st);
hipError_t launch_mlp_global_term(const Mlp &m, Workspace &ws, hipStream_t st);
hipError_t launch_mlp_items(Workspace &ws, hipStream_t st);
hipError_t launch_mlp_local(const Scene &sc, const Mlp &m, Workspace &ws, hipStream_t st);
hipError_t launch_mlp_pairs(const Scene &sc, const Mlp &m, Workspace &ws, hipStream_t st, bool far = false);
// adds the work items, pairs and slots of the list the pair kernels of this
// render consume (the same selection as theirs) to cnt[0..2]
hipError_t launch_count_items(Workspace &ws, bool far, unsigned long long *cnt, hipStream_t st);
bool mlp_fused_ok(const Scene &sc, const Mlp &m);
hipError_t launch_blend_fwd(Workspace &ws, float *C, bool save, hipStream_t st, bool redo = false);
hipError_t launch_far_items(Workspace &ws, hipStream_t st);
hipError_t launch_far_all(Workspace &ws, hipStream_t st);
int *far_count(Workspace &ws);
hipError_t launch_reduce_outputs(Workspace &ws, float *power, float *csum, hipStream_t st);
// backward (backward.hip)
hipError_t launch_blend_bwd(Workspace &ws, const float *C, const float *dC, const float *dP, const float *dA,
                            hipStream_t st);
// amp[j, p] = sqrt(Re^2 + Im^2 + AMP_EPS) of C (N x 2 x P) (kernels.hip)
hipError_t launch_amplitude(const float *C, float *amp, int N, size_t P, hipStream_t st);
// out[i] += add[i] for n floats (kernels.hip)
hipError_t launch_add_f32(float *out, const float *add, size_t n, hipStream_t st);
hipError_t launch_rad_bwd(const Scene &sc, Workspace &ws, float *grad, hipStream_t st);
hipError_t launch_mlp_bwd(const Scene &sc, const Mlp &m, Workspace &ws, float *gfeat, float *gmlp, hipStream_t st);
constexpr int PROJ_TERM_BYTES = 64;   // covariance upper triangle (6 doubles) and the mean (float4)
constexpr int PACC_STRIDE = 8;        // covariance terms (6), log2-opacity term, padding
hipError_t launch_project_bwd(const Scene &sc, Workspace &ws, const rxgs_grads &gr, hipStream_t st);
// deterministic backward (backward.hip)
int det_block_rows(const Workspace &ws);
hipError_t launch_det_gather(Workspace &ws, hipStream_t st);
hipError_t launch_live_rank(Workspace &ws, hipStream_t st);
size_t live_rank_words(const Workspace &ws);
hipError_t launch_det_rad(const Scene &sc, Workspace &ws, float *grad, int accum, hipStream_t st);
hipError_t launch_det_mlp_gather(Workspace &ws, hipStream_t st);
hipError_t launch_det_project(const Scene &sc, Workspace &ws, const rxgs_grads &gr, hipStream_t st);
size_t mlp_part_bytes(const Workspace &ws);
unsigned long long *stat_words(Workspace &ws);
int sort_items_for(uint32_t n);
size_t w1b_part_bytes(int64_t K);
size_t mlp_red_bytes();
hipError_t launch_blend_weights(Workspace &ws, hipStream_t st);
int *live_count(Workspace &ws);
size_t live_count_offset(const Workspace &ws);
// conditioned radiance (rxcond.hip): the receiver terms (no per-render
// counts needed), then the per-item local modulation and basis reduction
hipError_t launch_rxcond_receivers(const RxCond &m, Workspace &ws, hipStream_t st);
hipError_t launch_rxcond_pairs(const Scene &sc, const RxCond &m, Workspace &ws, hipStream_t st, bool far);
// upload steps: bounds of the means (6 order keys, preset by the caller to
// min = ~0, max = 0), the integer splat into acc (G^3 u64, zeroed), the
// occupancy values, the coefficients into walk order
hipError_t launch_rc_bounds(const Scene &sc, unsigned *keys, hipStream_t st);
float rc_key_value(unsigned key);
hipError_t launch_rc_splat(const Scene &sc, const RxCond &m, unsigned long long *acc, hipStream_t st);
hipError_t launch_rc_finish(const RxCond &m, const unsigned long long *acc, hipStream_t st);
hipError_t launch_rc_coef_perm(const float *src, int64_t K, const RxCond &m, hipStream_t st);
void release_rxcond(RxCond &m);

bool grow(DevBuf &b, size_t bytes, Allocator *al);
void release(DevBuf &b);

}  // namespace rxgs
