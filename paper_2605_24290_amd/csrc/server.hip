// Continuous-batching server of librxgs: a worker thread keeps the scene on
// the device, forms a batch from the queued queries whenever one of its slots
// (stream + workspace + pinned staging) is free, fuses the batch into one
// render (each query's transmitter is one view in TX mode) and retires the
// tickets when the slot's completion event fires.
#include "rxgs_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

using namespace rxgs;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int64_t round_up64(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

enum TicketState { T_QUEUED = 0, T_RUNNING = 1, T_DONE = 2, T_CANCELLED = 3, T_FAILED = 4 };

constexpr int MAX_ATTEMPTS = 2;   // a ticket rides at most this many batches (one replay)

struct Ticket {
    uint64_t id = 0;
    float tx[3] = {0, 0, 0};
    std::vector<float> rx;
    int n = 0;
    int state = T_QUEUED;
    int status = RXGS_OK;   // of a failed ticket
    int attempts = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int batch_q = 0, batch_n = 0;
    std::vector<float> power;
    std::vector<float> C;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    rxgs_saved *saved = nullptr;
    DevBuf d_tx, d_rx, d_C, d_P;
    float *h_in = nullptr;   // pinned: tx (Q x 3) then rx (N x 3)
    size_t h_in_cap = 0;
    float *h_P = nullptr;    // pinned: N
    size_t h_P_cap = 0;
    float *h_C = nullptr;    // pinned: N x 2 x H x W
    size_t h_C_cap = 0;
    bool busy = false;
    double t_launch = 0;
    std::vector<uint64_t> tickets;
    std::vector<int> offs;   // receiver offset of each ticket in the batch
    int N = 0;
    int64_t est_bytes = 0;   // admission estimate of the batch
    // host executor: results and completion of the batch in flight
    std::vector<float> host_P;
    double ready_at = 0;
    bool host_fail = false;
};

bool pinned_grow(float *&p, size_t &cap, size_t n)
{
    if (cap >= n) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const size_t want = std::max<size_t>(n + n / 4, 1024);
    if (hipHostMalloc((void **)&p, want * sizeof(float), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return false;
    }
    cap = want;
    return true;
}

// What runs the batches the scheduler forms: the GPU render, or a host-only
// stand-in for tests of the scheduling and failure paths.
struct Executor {
    virtual ~Executor() = default;
    virtual rxgs_status init_slot(rxgs_server *s, Slot &sl) = 0;
    virtual void free_slot(rxgs_server *s, Slot &sl) = 0;
    // enqueue one batch; on failure nothing of it is left in flight
    virtual rxgs_status launch(rxgs_server *s, Slot &sl, std::vector<Ticket *> &batch) = 0;
    // 0 finished, 1 still running, 2 failed
    virtual int query(Slot &sl) = 0;
    // results of ticket b of the slot's finished batch
    virtual void fetch(rxgs_server *s, Slot &sl, size_t b, Ticket &tk) = 0;
    // device memory the slot's last batch asked for (-1: not tracked)
    virtual int64_t used_bytes(rxgs_server *s, Slot &sl) = 0;
    // tile pairs per (view, Gaussian) of the slot's last batch (-1: not tracked)
    virtual double pairs_per_gaussian(Slot &sl) = 0;
};

}  // namespace

struct rxgs_server {
    rxgs_ctx *ctx = nullptr;   // NULL with the host executor
    Executor *exec = nullptr;
    rxgs_server_opts opts{};
    int64_t K = 0;
    int32_t H = 0, W = 0;
    int64_t slot_budget = 0;
    // tile pairs per (view, Gaussian) the admission estimate assumes: raised
    // to 1.25 x the largest ratio a render has shown
    double ppg = RXGS_EST_PAIRS_PER_GAUSSIAN;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Ticket> tickets;
    std::vector<Slot> slots;
    uint64_t next_id = 1;
    bool stopping = false;
    bool running = false;
    rxgs_server_stats_t st{};
    std::string err;
};

// ---------------------------------------------------------------------------
namespace {

int bits_of(uint64_t n)
{
    int b = 0;
    while ((1ull << b) < n) b++;
    return b;
}

// Upper bound of the device bytes one render of Q queries and N receivers asks
// for (the sum of its workspace buffer requests, as they are made in the
// render), plus the batch's inputs and outputs, given at most `ppg` tile pairs
// per (view, Gaussian) on average: the one quantity that depends on the scene.
int64_t estimate_bytes(int32_t mode, int32_t Q, int32_t N, int64_t K, int32_t H, int32_t W, double ppg)
{
    if (N <= 0) return 0;
    const bool tx = mode == RXGS_MODE_TX;
    const int64_t V = tx ? std::max(Q, 1) : N;
    const int64_t K1 = std::max<int64_t>(K, 1);
    const int64_t Kp = round_up64(K1, SORT_TILE);
    const int64_t VK = V * Kp;
    const int64_t P = (int64_t)H * W;
    const int64_t tiles = (int64_t)((H + TILE - 1) / TILE) * ((W + TILE - 1) / TILE);
    // tile pairs, each view's segment padded to whole sort units
    const int64_t Dpad = (int64_t)std::ceil(ppg * (double)V * (double)K1) + V * SORT_TILE;
    const uint32_t Dsort = (uint32_t)std::min<int64_t>(Dpad, 0xFFFFFFFFll);
    // MLP work items: per view ceil(visible / 32) x ceil(its receivers / 16),
    // and the sum over views of ceil(N_v / 16) is at most V + N / 16
    const int64_t items = (Kp / MLP_PAIRS) * (tx ? V + (N + MLP_RG - 1) / MLP_RG : V);
    int64_t b = 0;
    b += 4 * V + 12 * V + 12 * (int64_t)N;   // view flags; view centres and receivers (saved states)
    b += 72 * VK;                             // depth keys and values (two copies), records, boxes, order, pair offsets
    b += 52 * K1;                             // projection terms and cull bounds per Gaussian
    b += 4 * (4 * V + AMAX_SLOTS + 2 * STAT_WORDS + (int64_t)emit_word_count((int)V, Kp) + 16);   // counters
    b += (int64_t)sort_ws_bytes((uint32_t)std::min<int64_t>(VK, 0xFFFFFFFFll), 32, (int)V);    // depth sort
    b += 256 * (int64_t)N + 256 * K1;         // MLP layer-1 terms of the receivers and the Gaussians
    b += 16 * Dpad;                           // pair keys and values, two copies
    b += (int64_t)sort_ws_bytes(Dsort, std::max(bits_of((uint64_t)tiles), 1), (int)V);   // pair sort
    b += 12 * V * tiles;                      // tile ranges and tile order
    b += 8 * (int64_t)N * Kp;                 // radiance
    b += 8 * (tx ? V : (int64_t)N) * P;       // final transmittance, stop index
    b += 48 * (int64_t)N * tiles;             // per-sub-tile partial sums
    b += 3 * 16 * items;                      // work items: all, the live ones, those past the prefix
    b += 2 * (VK / MLP_PAIRS + 128);          // position-block marks (asked for by both TX paths)
    b += V * P * (FAR_RECORDS * 8 + 1) + 4 * V * tiles;   // far records of the radiance prefix, counts, sub-tile marks
    b += 4 * Dpad;                            // emission-order pair keys (deterministic saved states)
    b += 4 * VK + VK / 12 + 1040 * V + 64;    // direct binning: per-chunk tile counts, extents and units
    b += 20 * (int64_t)N + 80 * V + 16 * (Dpad / SORT_TILE + 1) + 1024;   // descriptors
    b += 12 * (int64_t)Q + 16 * (int64_t)N + 8 * (int64_t)N * P;   // transmitters, receivers, power, spectra
    return b;
}

int32_t plan_batch(const int32_t *n_rx, int32_t n_queued, int32_t mode, int64_t K, int32_t H, int32_t W,
                   int64_t budget_bytes, int32_t max_rx, int32_t max_queries, double ppg, int64_t *bytes_out)
{
    int32_t take = 0;
    int64_t total = 0, bytes = 0;
    if (n_rx && n_queued > 0)
        for (int32_t i = 0; i < n_queued && i < max_queries; i++) {
            const int64_t t2 = total + n_rx[i];
            if (n_rx[i] < 1 || t2 > max_rx) break;
            const int64_t b = estimate_bytes(mode, i + 1, (int32_t)t2, K, H, W, ppg);
            if (b > budget_bytes) break;
            take = i + 1;
            total = t2;
            bytes = b;
        }
    if (bytes_out) *bytes_out = bytes;
    return take;
}

}  // namespace

extern "C" int64_t rxgs_workspace_estimate(int32_t mode, int32_t Q, int32_t N, int64_t K, int32_t H, int32_t W)
{
    return estimate_bytes(mode, Q, N, K, H, W, RXGS_EST_PAIRS_PER_GAUSSIAN);
}

extern "C" int32_t rxgs_plan_batch(const int32_t *n_rx, int32_t n_queued, int32_t mode, int64_t K, int32_t H,
                                   int32_t W, int64_t budget_bytes, int32_t max_rx, int32_t max_queries,
                                   int64_t *bytes_out)
{
    return plan_batch(n_rx, n_queued, mode, K, H, W, budget_bytes, max_rx, max_queries, RXGS_EST_PAIRS_PER_GAUSSIAN,
                      bytes_out);
}

// ---------------------------------------------------------------------------
namespace {

// The GPU executor: one rxgs_render per batch on the slot's stream into its
// private workspace, results copied back to pinned memory.
struct GpuExecutor final : Executor {
    rxgs_status init_slot(rxgs_server *s, Slot &sl) override
    {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return RXGS_E_DEVICE;
        }
        if (rxgs_saved_create(s->ctx, &sl.saved) != RXGS_OK) return RXGS_E_OOM;
        sl.saved->keep = false;   // the slot's private workspace; nothing is kept for a backward
        return RXGS_OK;
    }

    void free_slot(rxgs_server *s, Slot &sl) override
    {
        (void)s;
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        (void)hipGetLastError();
        if (sl.saved) rxgs_saved_destroy(sl.saved);
        sl.saved = nullptr;
        release(sl.d_tx);
        release(sl.d_rx);
        release(sl.d_C);
        release(sl.d_P);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        sl.done = nullptr;
        sl.stream = nullptr;
    }

    rxgs_status launch(rxgs_server *s, Slot &sl, std::vector<Ticket *> &batch) override
    {
        rxgs_ctx *ctx = s->ctx;
        const int mode = s->opts.mode;
        const int Q = (int)batch.size();
        const int N = sl.N;
        const size_t P = (size_t)ctx->g.H * ctx->g.W;
        if (!pinned_grow(sl.h_in, sl.h_in_cap, (size_t)(Q + N) * 3) || !pinned_grow(sl.h_P, sl.h_P_cap, (size_t)N))
            return RXGS_E_OOM;
        if (s->opts.want_spectra && !pinned_grow(sl.h_C, sl.h_C_cap, (size_t)N * 2 * P)) return RXGS_E_OOM;
        std::vector<int32_t> rx_off(Q + 1, 0);
        for (int q = 0; q < Q; q++) {
            std::memcpy(sl.h_in + 3 * q, batch[q]->tx, 12);
            std::memcpy(sl.h_in + 3 * Q + 3 * sl.offs[q], batch[q]->rx.data(), (size_t)batch[q]->n * 12);
            rx_off[q + 1] = rx_off[q] + batch[q]->n;
        }
        rxgs::Allocator *al = &ctx->alloc;
        if (!grow(sl.d_tx, (size_t)Q * 12, al) || !grow(sl.d_rx, (size_t)N * 12, al) ||
            !grow(sl.d_P, (size_t)N * 4, al) || !grow(sl.d_C, (size_t)N * 2 * P * 4, al))
            return RXGS_E_OOM;
        if (hipMemcpyAsync(sl.d_tx.p, sl.h_in, (size_t)Q * 12, hipMemcpyHostToDevice, sl.stream) != hipSuccess ||
            hipMemcpyAsync(sl.d_rx.p, sl.h_in + 3 * Q, (size_t)N * 12, hipMemcpyHostToDevice, sl.stream) != hipSuccess) {
            (void)hipGetLastError();
            return RXGS_E_DEVICE;
        }
        rxgs_status rs = rxgs_render(ctx, mode, Q, sl.d_tx.as<float>(), rx_off.data(), N, sl.d_rx.as<float>(),
                                     sl.d_C.as<float>(), sl.d_P.as<float>(), nullptr, nullptr, sl.saved, sl.stream);
        if (rs != RXGS_OK) return rs;
        if (hipMemcpyAsync(sl.h_P, sl.d_P.p, (size_t)N * 4, hipMemcpyDeviceToHost, sl.stream) != hipSuccess) {
            (void)hipGetLastError();
            return RXGS_E_DEVICE;
        }
        if (s->opts.want_spectra &&
            hipMemcpyAsync(sl.h_C, sl.d_C.p, (size_t)N * 2 * P * 4, hipMemcpyDeviceToHost, sl.stream) != hipSuccess) {
            (void)hipGetLastError();
            return RXGS_E_DEVICE;
        }
        if (hipEventRecord(sl.done, sl.stream) != hipSuccess) {
            (void)hipGetLastError();
            return RXGS_E_DEVICE;
        }
        return RXGS_OK;
    }

    int query(Slot &sl) override
    {
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) return 1;
        if (q == hipSuccess) return 0;
        (void)hipGetLastError();
        return 2;
    }

    void fetch(rxgs_server *s, Slot &sl, size_t b, Ticket &tk) override
    {
        const size_t P = (size_t)s->ctx->g.H * s->ctx->g.W;
        tk.power.assign(sl.h_P + sl.offs[b], sl.h_P + sl.offs[b] + tk.n);
        if (s->opts.want_spectra)
            tk.C.assign(sl.h_C + (size_t)sl.offs[b] * 2 * P, sl.h_C + (size_t)(sl.offs[b] + tk.n) * 2 * P);
    }

    int64_t used_bytes(rxgs_server *s, Slot &sl) override
    {
        if (!sl.saved) return -1;
        const int64_t P = (int64_t)s->H * s->W;
        // the workspace buffers the render asked for, and the batch's inputs and outputs
        return (int64_t)sl.saved->ws.req_bytes + (int64_t)sl.tickets.size() * 12 + (int64_t)sl.N * 16 +
               (int64_t)sl.N * 2 * P * 4;
    }

    double pairs_per_gaussian(Slot &sl) override
    {
        const rxgs::Workspace &w = sl.saved->ws;
        return (w.V > 0 && w.K > 0) ? (double)w.D / ((double)w.V * (double)w.K) : -1.0;
    }
};

// The host executor: every batch "renders" power_j = tx.x + r.x + 2 r.y + 3 r.z
// per receiver after a fixed delay; launches and completions fail as scripted.
struct HostExecutor final : Executor {
    rxgs_host_executor cfg{};
    int64_t launches = 0;

    rxgs_status init_slot(rxgs_server *, Slot &) override { return RXGS_OK; }
    void free_slot(rxgs_server *, Slot &sl) override { sl.host_P.clear(); }

    rxgs_status launch(rxgs_server *, Slot &sl, std::vector<Ticket *> &batch) override
    {
        const int64_t i = launches++;
        const uint64_t bit = i < 64 ? (1ull << i) : 0ull;
        if (cfg.fail_launch_mask & bit) return RXGS_E_OOM;
        sl.host_P.assign(sl.N, 0.f);
        for (size_t q = 0; q < batch.size(); q++)
            for (int j = 0; j < batch[q]->n; j++) {
                const float *r = batch[q]->rx.data() + 3 * j;
                sl.host_P[sl.offs[q] + j] = batch[q]->tx[0] + r[0] + 2.f * r[1] + 3.f * r[2];
            }
        sl.host_fail = (cfg.fail_device_mask & bit) != 0;
        sl.ready_at = now_s() + 1e-6 * cfg.delay_us;
        return RXGS_OK;
    }

    int query(Slot &sl) override
    {
        if (now_s() < sl.ready_at) return 1;
        return sl.host_fail ? 2 : 0;
    }

    void fetch(rxgs_server *, Slot &sl, size_t b, Ticket &tk) override
    {
        tk.power.assign(sl.host_P.begin() + sl.offs[b], sl.host_P.begin() + sl.offs[b] + tk.n);
    }

    int64_t used_bytes(rxgs_server *, Slot &) override { return -1; }
    double pairs_per_gaussian(Slot &) override { return -1.0; }
};

// a batch that failed (at launch or on the device): the slot is made again
// and each of its tickets goes back to the front of the queue, once; a ticket
// whose second batch fails is retired with the failure
void batch_failed(rxgs_server *s, Slot &sl, rxgs_status why)
{
    s->st.failed_batches++;
    s->exec->free_slot(s, sl);
    if (s->exec->init_slot(s, sl) != RXGS_OK) s->err = "slot could not be made again after a failed batch";
    const double t = now_s();
    for (size_t b = sl.tickets.size(); b-- > 0;) {
        auto it = s->tickets.find(sl.tickets[b]);
        if (it == s->tickets.end()) continue;
        Ticket &tk = it->second;
        if (tk.attempts < MAX_ATTEMPTS && !s->stopping) {
            tk.state = T_QUEUED;
            s->queue.push_front(tk.id);
            s->st.queued++;
            s->st.replayed++;
        } else {
            tk.state = T_FAILED;
            tk.status = why;
            tk.t_done = t;
            s->st.failed++;
        }
    }
    s->st.in_flight -= (int64_t)sl.tickets.size();
    sl.tickets.clear();
    sl.busy = false;
    s->cv_done.notify_all();
}

void worker_main(rxgs_server *s)
{
    if (s->ctx) (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // retire finished batches
        bool any_busy = false;
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            const int q = s->exec->query(sl);
            if (q == 1) {
                any_busy = true;
                continue;
            }
            if (q == 2) {
                s->st.busy_s += now_s() - sl.t_launch;
                batch_failed(s, sl, RXGS_E_DEVICE);
                continue;
            }
            const double t = now_s();
            for (size_t b = 0; b < sl.tickets.size(); b++) {
                auto it = s->tickets.find(sl.tickets[b]);
                if (it == s->tickets.end()) continue;
                Ticket &tk = it->second;
                s->exec->fetch(s, sl, b, tk);
                tk.state = T_DONE;
                tk.t_done = t;
                s->st.completed++;
            }
            s->st.busy_s += t - sl.t_launch;
            s->st.in_flight -= (int64_t)sl.tickets.size();
            sl.tickets.clear();
            sl.busy = false;
            s->cv_done.notify_all();
        }
        if (s->stopping && !any_busy) {
            bool busy_now = false;
            for (Slot &sl : s->slots) busy_now |= sl.busy;
            if (!busy_now) break;
        }
        // launch batches on free slots (continuous batching)
        bool launched = false;
        if (!s->stopping) {
            for (Slot &sl : s->slots) {
                if (sl.busy || s->queue.empty()) continue;
                std::vector<int32_t> ns;
                for (size_t i = 0; i < s->queue.size() && (int)i < s->opts.max_queries_per_batch; i++)
                    ns.push_back(s->tickets[s->queue[i]].n);
                int64_t bytes = 0;
                const int take = plan_batch(ns.data(), (int32_t)ns.size(), s->opts.mode, s->K, s->H, s->W,
                                            s->slot_budget, s->opts.max_rx_per_batch, s->opts.max_queries_per_batch,
                                            s->ppg, &bytes);
                if (take < 1) break;
                std::vector<Ticket *> batch;
                sl.tickets.clear();
                sl.offs.clear();
                int nrx = 0;
                const double t = now_s();
                for (int i = 0; i < take; i++) {
                    Ticket &tk = s->tickets[s->queue.front()];
                    s->queue.pop_front();
                    tk.state = T_RUNNING;
                    tk.t_start = t;
                    tk.attempts++;
                    batch.push_back(&tk);
                    sl.tickets.push_back(tk.id);
                    sl.offs.push_back(nrx);
                    nrx += tk.n;
                }
                for (Ticket *tk : batch) {
                    tk->batch_q = take;
                    tk->batch_n = nrx;
                }
                sl.N = nrx;
                sl.est_bytes = bytes;
                s->st.queued -= take;
                s->st.in_flight += take;
                s->st.batches++;
                s->st.receivers += nrx;
                sl.busy = true;
                sl.t_launch = t;
                // ticket storage is stable while running (only this thread erases running tickets)
                lk.unlock();
                const rxgs_status rs = s->exec->launch(s, sl, batch);
                const int64_t used = rs == RXGS_OK ? s->exec->used_bytes(s, sl) : -1;
                const double ppg = rs == RXGS_OK ? s->exec->pairs_per_gaussian(sl) : -1.0;
                lk.lock();
                if (rs != RXGS_OK) {
                    if (s->ctx) s->err = s->ctx->err;
                    batch_failed(s, sl, rs);
                } else if (used >= 0) {
                    s->st.peak_slot_bytes = std::max(s->st.peak_slot_bytes, used);
                    if (used > sl.est_bytes) s->st.over_estimate++;
                }
                if (ppg > 0.0) s->ppg = std::max(s->ppg, 1.25 * ppg);
                launched = true;
            }
        }
        if (launched) continue;
        bool busy_now = false;
        for (Slot &sl : s->slots) busy_now |= sl.busy;
        if (busy_now)
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
    s->running = false;
}

rxgs_status server_options_ok(const rxgs_server_opts *opts)
{
    if (opts->max_rx_per_batch < 1 || opts->max_queries_per_batch < 1 || opts->slots < 1 || opts->slots > 8 ||
        (opts->mode != RXGS_MODE_TX && opts->mode != RXGS_MODE_RX) || opts->queue_capacity < 1 ||
        opts->mem_budget_bytes < 0)
        return RXGS_E_INVALID;
    return RXGS_OK;
}

// slots made by the executor, then the worker started
rxgs_status start_worker(rxgs_server *s)
{
    s->slot_budget = s->opts.mem_budget_bytes / s->opts.slots;
    s->slots.resize(s->opts.slots);
    for (Slot &sl : s->slots) {
        const rxgs_status rs = s->exec->init_slot(s, sl);
        if (rs != RXGS_OK) return rs;
    }
    s->running = true;
    s->worker = std::thread(worker_main, s);
    return RXGS_OK;
}

}  // namespace

extern "C" rxgs_status rxgs_server_start(rxgs_ctx *ctx, const rxgs_server_opts *opts, rxgs_server **out)
{
    if (!ctx || !opts || !out) return RXGS_E_INVALID;
    *out = nullptr;
    if (server_options_ok(opts) != RXGS_OK) {
        ctx->err = "invalid server options";
        return RXGS_E_INVALID;
    }
    if (!ctx->scene.valid || (ctx->scene.has_features && !ctx->mlp.valid) || ctx->scene.geometry_only) {
        ctx->err = "server needs an uploaded scene (and MLP)";
        return RXGS_E_STATE;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        (void)hipGetLastError();
        return RXGS_E_DEVICE;
    }
    rxgs_server *s = new (std::nothrow) rxgs_server();
    if (!s) return RXGS_E_OOM;
    s->ctx = ctx;
    s->exec = new (std::nothrow) GpuExecutor();
    if (!s->exec) {
        delete s;
        return RXGS_E_OOM;
    }
    s->opts = *opts;
    s->K = ctx->scene.K;
    s->H = ctx->g.H;
    s->W = ctx->g.W;
    if (s->opts.mem_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            fr = (size_t)8 << 30;
        }
        s->opts.mem_budget_bytes = (int64_t)(fr / 2);
    }
    const rxgs_status rs = start_worker(s);
    if (rs != RXGS_OK) {
        ctx->err = "server slot creation failed";
        rxgs_server_stop(s);
        return rs;
    }
    *out = s;
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_server_start_host(const rxgs_server_opts *opts, const rxgs_host_executor *exec,
                                              rxgs_server **out)
{
    if (!opts || !exec || !out) return RXGS_E_INVALID;
    *out = nullptr;
    if (server_options_ok(opts) != RXGS_OK || opts->want_spectra || opts->mem_budget_bytes <= 0 || exec->K < 0 ||
        exec->H < 1 || exec->W < 1 || exec->delay_us < 0)
        return RXGS_E_INVALID;
    rxgs_server *s = new (std::nothrow) rxgs_server();
    if (!s) return RXGS_E_OOM;
    HostExecutor *he = new (std::nothrow) HostExecutor();
    if (!he) {
        delete s;
        return RXGS_E_OOM;
    }
    he->cfg = *exec;
    s->exec = he;
    s->opts = *opts;
    s->K = exec->K;
    s->H = exec->H;
    s->W = exec->W;
    const rxgs_status rs = start_worker(s);
    if (rs != RXGS_OK) {
        rxgs_server_stop(s);
        return rs;
    }
    *out = s;
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_server_submit(rxgs_server *s, const float *tx, int32_t n, const float *rx_host,
                                          uint64_t *ticket)
{
    if (!s || !tx || !rx_host || !ticket || n < 1) return RXGS_E_INVALID;
    if (n > s->opts.max_rx_per_batch) return RXGS_E_INVALID;
    for (int i = 0; i < 3; i++)
        if (!std::isfinite(tx[i])) return RXGS_E_INVALID;
    for (int64_t i = 0; i < 3 * (int64_t)n; i++)
        if (!std::isfinite(rx_host[i])) return RXGS_E_INVALID;
    if (estimate_bytes(s->opts.mode, 1, n, s->K, s->H, s->W, s->ppg) > s->slot_budget) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->st.rejected++;
        return RXGS_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping || !s->running) return RXGS_E_STATE;
    if ((int64_t)s->queue.size() >= s->opts.queue_capacity) {
        s->st.rejected++;
        return RXGS_E_BUSY;
    }
    Ticket tk;
    tk.id = s->next_id++;
    std::memcpy(tk.tx, tx, 12);
    tk.rx.assign(rx_host, rx_host + 3 * (size_t)n);
    tk.n = n;
    tk.t_submit = now_s();
    const uint64_t id = tk.id;
    s->tickets.emplace(id, std::move(tk));
    s->queue.push_back(id);
    s->st.submitted++;
    s->st.queued++;
    *ticket = id;
    s->cv_work.notify_one();
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_server_poll(rxgs_server *s, uint64_t ticket, float *power_host, float *C_host,
                                        rxgs_ticket_info *info, int32_t timeout_ms)
{
    if (!s) return RXGS_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return RXGS_E_INVALID;
    auto ready = [&] {
        auto i2 = s->tickets.find(ticket);
        return i2 == s->tickets.end() || i2->second.state >= T_DONE;
    };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        return RXGS_E_TIMEOUT;
    it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return RXGS_E_INVALID;
    Ticket &tk = it->second;
    rxgs_status rs = RXGS_OK;
    if (tk.state == T_CANCELLED) rs = RXGS_E_CANCELLED;
    else if (tk.state == T_FAILED) rs = tk.status == RXGS_OK ? RXGS_E_DEVICE : (rxgs_status)tk.status;
    else {
        if (power_host) std::memcpy(power_host, tk.power.data(), tk.power.size() * 4);
        if (C_host && !tk.C.empty()) std::memcpy(C_host, tk.C.data(), tk.C.size() * 4);
    }
    if (info) {
        info->t_submit = tk.t_submit;
        info->t_start = tk.t_start;
        info->t_done = tk.t_done;
        info->batch_queries = tk.batch_q;
        info->batch_receivers = tk.batch_n;
        info->attempts = tk.attempts;
        info->reserved = 0;
    }
    s->tickets.erase(it);
    return rs;
}

extern "C" rxgs_status rxgs_server_cancel(rxgs_server *s, uint64_t ticket)
{
    if (!s) return RXGS_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return RXGS_E_INVALID;
    if (it->second.state != T_QUEUED) return RXGS_E_STATE;
    auto q = std::find(s->queue.begin(), s->queue.end(), ticket);
    if (q != s->queue.end()) s->queue.erase(q);
    it->second.state = T_CANCELLED;
    it->second.t_done = now_s();
    s->st.cancelled++;
    s->st.queued--;
    s->cv_done.notify_all();
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_server_stats(rxgs_server *s, rxgs_server_stats_t *out)
{
    if (!s || !out) return RXGS_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return RXGS_OK;
}

extern "C" rxgs_status rxgs_server_stop(rxgs_server *s)
{
    if (!s) return RXGS_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (uint64_t id : s->queue) {
            auto it = s->tickets.find(id);
            if (it != s->tickets.end()) {
                it->second.state = T_CANCELLED;
                s->st.cancelled++;
            }
        }
        s->queue.clear();
        s->st.queued = 0;
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    if (s->ctx) (void)hipSetDevice(s->ctx->device);
    for (Slot &sl : s->slots) {
        if (s->exec) s->exec->free_slot(s, sl);
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.h_P) (void)hipHostFree(sl.h_P);
        if (sl.h_C) (void)hipHostFree(sl.h_C);
    }
    delete s->exec;
    delete s;
    return RXGS_OK;
}
