// Serving runtime: continuous batching of scan requests on one GPU.
//
// Requests are admitted in FIFO order against a device-memory arena (outputs
// and node tables) and a slot table.  A scheduler thread repeatedly packs wave
// tiles of every running request into persistent kernel launches (one per
// precision x lanes-per-point group), giving each running request a fair share
// of the batch's evaluation budget.  Within a launch the most expensive tiles
// are handed out first, so the launch ends on short ones.  A batch's staging
// copy, table uploads and subtraction sums run on a prologue stream; its
// launches run on compute streams taken in turn, each waiting for its own
// prologue only, so the waves of the next batch (and of the other precision)
// fill the compute units that a launch's last long tiles leave idle.  Three
// batches stay in flight so the GPU never waits for the host.  A request is
// done when its last tile's batch has completed (HIP events); its output stays
// in the arena until released.
//
// Every point is computed by the same device function, table values and
// subtraction-sum kernel as a standalone scan with one lane per point, so a
// served result is bitwise identical to gf_scan_plan_ex(..., 1, ...) and does
// not depend on what else was in flight.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/gf.h"
#include "gf_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over a device arena: free ranges in an offset-ordered
// map, coalesced on release; 256-byte granules.
class Arena {
public:
    void init(size_t size)
    {
        size_ = size;
        free_.clear();
        free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = gf::align256(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, noff = it->first + bytes;
            free_.erase(it);
            if (rest) free_[noff] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = gf::align256(std::max<size_t>(bytes, 1));
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

// A node table resident in the arena, shared by requests with the same key.
struct Table {
    size_t off = 0, bytes = 0;
    int refs = 0;
    std::vector<char> host;  // contents, uploaded through a staging buffer
    bool uploaded = false;
    double wmid = 0.0;       // angular tables: middle-node weight
    size_t off32 = 0;        // angular tables: offset of the FP32 pair table
};

struct Request {
    uint64_t ticket = 0;
    gf_params p{};
    gf_grid g{};
    gf_quadrature q{};
    gf_propagators props{};
    bool has_props = false;
    int state = GF_REQ_QUEUED;
    int slot = -1;
    size_t out_off = 0, out_bytes = 0;
    std::string keys[3];  // radial, angular, arc table keys
    int lanes = 1;
    long long n_tiles = 0, next_tile = 0, tiles_done = 0;
    double cost_per_tile = 0.0;
    Clock::time_point t_submit, t_done;
    gf::ScanArgs args{};
};

// Host-pinned staging buffer and its device twin, reused after its batch's
// event has completed.
struct Stage {
    char *h = nullptr;
    char *d = nullptr;
    size_t bytes = 0, used = 0;
    void *bump(size_t n, size_t *doff)
    {
        size_t off = gf::align256(used);
        if (off + n > bytes) return nullptr;
        used = off + n;
        *doff = off;
        return h + off;
    }
};

// A table upload staged in this iteration: stage offset -> arena offset.
struct Upload {
    size_t stage_off, arena_off, bytes;
};

struct Batch {
    std::vector<hipEvent_t> ev;  // all must complete
    int stage = 0;
    std::vector<std::pair<Request *, long long>> tiles;  // tiles per request
    long long items = 0;
};

constexpr int kMaxInflight = 3;
constexpr int kStages = kMaxInflight + 1;  // one per batch in flight + the one being filled
constexpr int kComputeStreams = 2;
constexpr int kMaxGroups = 8;  // precision x split x pole sums (one lanes value)
constexpr size_t kStageBytes = 32u << 20;
constexpr long long kMaxItemsPerBatch = 1 << 20;
constexpr int kMaxNewPerBatch = 256;

}  // namespace

struct gf_server {
    int device = -1;
    gf_server_config cfg{};
    hipStream_t stream = nullptr;           // prologue: staging, uploads, subtraction sums
    hipStream_t comp[kComputeStreams] = {};  // persistent serve launches, in turn
    int next_comp = 0;
    hipEvent_t group_ev[kStages][kMaxGroups] = {};
    std::map<std::tuple<int, int, int, int>, int> resident;  // waves per launch group
    // items a batch takes at least while tiles remain: between fill_min and
    // fill_max, half the tiles still to run
    long long fill_min = 0, fill_max = 0;
    char *d_arena = nullptr;
    Arena arena;
    gf::ScanArgs *d_args = nullptr;
    double *d_jmu = nullptr;
    Stage stage[kStages];
    hipEvent_t stage_ev[kStages] = {};
    int next_stage = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::vector<Request *> running;  // admission order
    std::unordered_map<uint64_t, Request *> reqs;
    std::deque<uint64_t> completed;  // done, not yet reported by wait_any
    std::vector<int> free_slots;
    std::map<std::string, Table> tables;
    std::thread worker;
    bool stop = false;
    bool admit_blocked = false;  // the queue head did not fit; retry after a release
    int worker_error = GF_OK;
    std::string worker_msg;
    uint64_t next_ticket = 1;

    // statistics
    int64_t n_submitted = 0, n_completed = 0, n_released = 0, n_rejected = 0;
    int64_t n_batches = 0, n_items = 0, points_done = 0;
    double nominal_evals = 0.0;
    std::vector<double> latencies_ms;
    bool any_submit = false;
    Clock::time_point first_submit, last_done;

    void run();
    bool admit_one(Request *r, Stage &st, std::vector<Request *> &fresh,
                   std::vector<Upload> &uploads);
    Table *ensure_table(const std::string &key, const Request &r, bool *fits);
    void finish(Request *r);
    int fail_worker(hipError_t e, const char *what);
};

namespace {

std::string key_radial(const gf_quadrature &q, const gf_params &p)
{
    std::string k = "r" + std::to_string(q.n_radial) + ":" +
                    std::to_string(p.dimension == 0 ? 4 : p.dimension) + ":" +
                    std::to_string(q.radial_split) + ":";
    k.append(reinterpret_cast<const char *>(&p.lambda2), sizeof(double));
    return k;
}
std::string key_angular(const gf_quadrature &q, const gf_params &p)
{
    return "a" + std::to_string(q.n_angular) + ":" + std::to_string(q.angular_rule) + ":" +
           std::to_string(p.dimension == 0 ? 4 : p.dimension);
}
std::string key_arc(const gf_quadrature &q) { return "c" + std::to_string(q.n_arc); }

// Arena bytes of a request's three node tables, as ensure_table builds them:
// radial [r | sqrt r | W] (3 n_r doubles), angular pairs in FP64 then FP32
// (3 max(n_a/2, 1) each), arc [xi | w] (2 n_arc doubles); each range is
// rounded up to the arena's 256-byte granule.
size_t table_bytes(const gf_quadrature &q)
{
    const size_t npair = (size_t)std::max(q.n_angular / 2, 1);
    const size_t rad = 3 * (size_t)q.n_radial * sizeof(double);
    const size_t ang = gf::align256(3 * npair * sizeof(double)) + 3 * npair * sizeof(float);
    const size_t arc = 2 * (size_t)std::max(q.n_arc, 1) * sizeof(double);
    return gf::align256(rad) + gf::align256(ang) + gf::align256(arc);
}

double nominal_evals_per_point(const gf_quadrature &q)
{
    return (double)(q.n_radial + q.n_arc) * (double)q.n_angular;
}

}  // namespace

int gf_server::fail_worker(hipError_t e, const char *what)
{
    std::lock_guard<std::mutex> lock(mu);
    worker_error = GF_EDEVICE;
    worker_msg = std::string(what) + ": " + hipGetErrorString(e);
    stop = true;
    cv_done.notify_all();
    return GF_EDEVICE;
}

// Builds (or finds) a table in the arena; *fits = false if it cannot be
// placed now.  Called with the lock held.
Table *gf_server::ensure_table(const std::string &key, const Request &r, bool *fits)
{
    *fits = true;
    auto it = tables.find(key);
    if (it != tables.end()) return &it->second;
    Table t;
    if (key[0] == 'r') {
        std::vector<double> rad;
        gf::radial_table(r.q.n_radial, r.p.lambda2, r.p.dimension == 0 ? 4 : r.p.dimension,
                         r.q.radial_split, rad);
        t.host.resize(rad.size() * sizeof(double));
        std::memcpy(t.host.data(), rad.data(), t.host.size());
    } else if (key[0] == 'a') {
        std::vector<double> ang;
        std::vector<float> ang32;
        gf::angular_tables(r.q.n_angular, r.q.angular_rule, r.p.dimension == 0 ? 4 : r.p.dimension,
                           ang, ang32, &t.wmid);
        const size_t b64 = gf::align256(ang.size() * sizeof(double));
        t.host.assign(b64 + ang32.size() * sizeof(float), 0);
        std::memcpy(t.host.data(), ang.data(), ang.size() * sizeof(double));
        std::memcpy(t.host.data() + b64, ang32.data(), ang32.size() * sizeof(float));
        t.off32 = b64;
    } else {
        std::vector<double> arc;
        gf::arc_table(r.q.n_arc, arc);
        t.host.resize(arc.size() * sizeof(double));
        std::memcpy(t.host.data(), arc.data(), t.host.size());
    }
    t.bytes = t.host.size();
    if (!arena.alloc(t.bytes, &t.off)) {
        // evict unreferenced tables and retry once
        for (auto jt = tables.begin(); jt != tables.end();) {
            if (jt->second.refs == 0) {
                arena.release(jt->second.off, jt->second.bytes);
                jt = tables.erase(jt);
            } else {
                ++jt;
            }
        }
        if (!arena.alloc(t.bytes, &t.off)) {
            *fits = false;
            return nullptr;
        }
    }
    auto res = tables.emplace(key, std::move(t));
    return &res.first->second;
}

// Admits one request if its output and tables fit; stages its argument record
// and any table upload.  Called with the lock held.
bool gf_server::admit_one(Request *r, Stage &st, std::vector<Request *> &fresh,
                          std::vector<Upload> &uploads)
{
    if (free_slots.empty()) return false;
    size_t out_off;
    if (!arena.alloc(r->out_bytes, &out_off)) {
        for (auto jt = tables.begin(); jt != tables.end();) {
            if (jt->second.refs == 0) {
                arena.release(jt->second.off, jt->second.bytes);
                jt = tables.erase(jt);
            } else {
                ++jt;
            }
        }
        if (!arena.alloc(r->out_bytes, &out_off)) return false;
    }
    // Each table is pinned (refs raised) as soon as it is found or built, so
    // that building the next one cannot evict it; every failure below unpins
    // what this call pinned and returns the output range.
    Table *tb[3] = {nullptr, nullptr, nullptr};
    auto undo = [&](int pinned) {
        for (int k = 0; k < pinned; ++k) --tb[k]->refs;
        arena.release(out_off, r->out_bytes);
        return false;
    };
    for (int k = 0; k < 3; ++k) {
        bool fits;
        tb[k] = ensure_table(r->keys[k], *r, &fits);
        if (!fits) return undo(k);
        ++tb[k]->refs;
    }
    // staging space for new table contents: reserved for all of them before
    // any is marked uploaded, so a failed admission stages nothing
    size_t need = st.used;
    for (int k = 0; k < 3; ++k)
        if (!tb[k]->uploaded) need = gf::align256(need) + tb[k]->bytes;
    if (need > st.bytes) return undo(3);
    for (int k = 0; k < 3; ++k) {
        if (tb[k]->uploaded) continue;
        size_t doff;
        void *h = st.bump(tb[k]->bytes, &doff);
        std::memcpy(h, tb[k]->host.data(), tb[k]->bytes);
        uploads.push_back(Upload{doff, tb[k]->off, tb[k]->bytes});
        tb[k]->uploaded = true;
    }
    r->out_off = out_off;
    r->slot = free_slots.back();
    free_slots.pop_back();
    gf::ScanArgs &a = r->args;
    gf::fill_constants(a, r->p, r->has_props ? &r->props : nullptr, r->q);
    a.rad = reinterpret_cast<const double *>(d_arena + tb[0]->off);
    a.ang = reinterpret_cast<const double *>(d_arena + tb[1]->off);
    a.ang32 = reinterpret_cast<const float *>(d_arena + tb[1]->off + tb[1]->off32);
    a.wmid = tb[1]->wmid;
    a.arc = reinterpret_cast<const double *>(d_arena + tb[2]->off);
    a.jmu = d_jmu + 2 * (GF_MAX_TAYLOR + 1) * (size_t)r->slot;
    // cannot fail: one lane per point on a grid checked at submission (at
    // most 2^31 points, 2^25 tiles)
    (void)gf::set_grid(a, r->g, r->lanes);
    a.out = reinterpret_cast<double *>(d_arena + out_off);
    a.cls = nullptr;
    r->n_tiles = a.n_tiles;
    r->state = GF_REQ_RUNNING;
    fresh.push_back(r);
    return true;
}

void gf_server::finish(Request *r)
{
    r->state = GF_REQ_DONE;
    r->t_done = Clock::now();
    last_done = r->t_done;
    latencies_ms.push_back(
        std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
    ++n_completed;
    points_done += (int64_t)r->g.n_re * r->g.n_im;
    nominal_evals += (double)r->g.n_re * r->g.n_im * nominal_evals_per_point(r->q);
    completed.push_back(r->ticket);
}

void gf_server::run()
{
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        fail_worker(e, "hipSetDevice");
        return;
    }
    std::deque<Batch> inflight;
    for (;;) {
        Batch b;
        std::vector<Request *> fresh;
        std::vector<Upload> uploads;
        // launch groups: (precision, lanes per point, split radial rule, pole sums)
        // -> runs of consecutive tiles (request, first tile, count)
        std::map<std::tuple<int, int, int, int>, std::vector<std::tuple<Request *, long long, long long>>>
            runs;
        std::map<std::tuple<int, int, int, int>, std::vector<gf::WorkItem>> groups;
        Stage &st = stage[next_stage];
        {
            std::unique_lock<std::mutex> lock(mu);
            if (inflight.empty()) {
                cv_work.wait_for(lock, std::chrono::milliseconds(2), [&] {
                    if (stop || (!pending.empty() && !admit_blocked)) return true;
                    for (Request *r : running)
                        if (r->next_tile < r->n_tiles) return true;
                    return false;
                });
            }
            if (stop && inflight.empty()) break;
            st.used = 0;
            // admission, FIFO
            while (!stop && !pending.empty() && (int)fresh.size() < kMaxNewPerBatch) {
                Request *r = pending.front();
                if (!admit_one(r, st, fresh, uploads)) {
                    admit_blocked = true;
                    break;
                }
                pending.pop_front();
                running.push_back(r);
            }
            // batch: fair share of the evaluation budget, oldest first
            std::vector<Request *> active;
            if (!stop)
                for (Request *r : running)
                    if (r->next_tile < r->n_tiles) active.push_back(r);
            if (!active.empty()) {
                // top-up target: 1.5 rounds of resident waves while little work
                // waits (short batches keep latency low), growing with the
                // backlog to 6 rounds (long launches amortise their drain and
                // the per-batch costs under load)
                long long backlog = 0;
                for (Request *r : active) backlog += r->n_tiles - r->next_tile;
                const long long fill_items = std::min(fill_max, std::max(fill_min, backlog / 2));
                // first pass: each request's share of the budget grows with the
                // square of its age (ms since submission + 1), so requests that
                // have waited long catch up with the ones that arrived after
                // them (at 80 % load the p99 latency 46 -> 39 ms, p50 19 -> 16 ms
                // against equal shares, same throughput; unchanged at 50 %);
                // second pass: what is left, oldest first
                double budget = cfg.batch_evals;
                const auto now = Clock::now();
                auto age2 = [&](const Request *r) {
                    const double a = 1.0 + std::chrono::duration<double, std::milli>(now - r->t_submit).count();
                    return a * a;
                };
                double age2_sum = 0.0;
                for (Request *r : active) age2_sum += age2(r);
                const double budget0 = budget;
                for (int pass = 0; pass < 2 && budget > 0.0 && b.items < kMaxItemsPerBatch;
                     ++pass) {
                    for (Request *r : active) {
                        long long left = r->n_tiles - r->next_tile;
                        if (left <= 0) continue;
                        double want = pass == 0 ? budget0 * age2(r) / age2_sum : budget;
                        long long k = (long long)std::ceil(want / r->cost_per_tile);
                        k = std::max(1LL, std::min(k, left));
                        k = std::min(k, kMaxItemsPerBatch - b.items);
                        if (k <= 0) break;
                        runs[{r->q.precision, r->lanes, r->q.radial_split, r->has_props ? 1 : 0}]
                            .emplace_back(r, r->next_tile, k);
                        r->next_tile += k;
                        b.tiles.emplace_back(r, k);
                        b.items += k;
                        budget -= (double)k * r->cost_per_tile;
                        if (budget <= 0.0 || b.items >= kMaxItemsPerBatch) break;
                    }
                }
                // the budget bought too few (long) tiles to occupy every wave
                // slot: top up, oldest first, so the launch is not one short
                // of work while tiles remain
                for (Request *r : active) {
                    if (b.items >= fill_items) break;
                    const long long k = std::min(r->n_tiles - r->next_tile, fill_items - b.items);
                    if (k <= 0) continue;
                    runs[{r->q.precision, r->lanes, r->q.radial_split, r->has_props ? 1 : 0}]
                        .emplace_back(r, r->next_tile, k);
                    r->next_tile += k;
                    b.tiles.emplace_back(r, k);
                    b.items += k;
                }
            }
        }

        // longest tiles first within each launch (stable: ties keep admission order)
        for (auto &kv : runs) {
            auto &rv = kv.second;
            std::stable_sort(rv.begin(), rv.end(), [](const auto &x, const auto &y) {
                return std::get<0>(x)->cost_per_tile > std::get<0>(y)->cost_per_tile;
            });
            auto &vec = groups[kv.first];
            for (const auto &run : rv)
                for (long long t = 0; t < std::get<2>(run); ++t)
                    vec.push_back(gf::WorkItem{std::get<0>(run)->slot,
                                               (int32_t)(std::get<1>(run) + t)});
        }

        if (groups.size() > (size_t)kMaxGroups) {
            fail_worker(hipErrorInvalidValue, "too many launch groups in one batch");
            break;
        }
        const bool launch_now = !fresh.empty() || b.items > 0;
        if (launch_now) {
            // stage: argument records, subtraction-sum inputs, counters, items
            size_t off_args = 0, off_slots = 0, off_mu2 = 0, off_cnt = 0;
            gf::ScanArgs *h_args = static_cast<gf::ScanArgs *>(
                st.bump(std::max<size_t>(1, fresh.size()) * sizeof(gf::ScanArgs), &off_args));
            int *h_slots = static_cast<int *>(
                st.bump(std::max<size_t>(1, fresh.size()) * sizeof(int), &off_slots));
            double *h_mu2 = static_cast<double *>(
                st.bump(std::max<size_t>(1, fresh.size()) * sizeof(double), &off_mu2));
            unsigned *h_cnt = static_cast<unsigned *>(
                st.bump(std::max<size_t>(1, groups.size()) * sizeof(unsigned), &off_cnt));
            std::vector<size_t> off_items;
            bool ok = h_args && h_slots && h_mu2 && h_cnt;
            for (auto &kv : groups) {
                size_t o = 0;
                void *h = ok ? st.bump(kv.second.size() * sizeof(gf::WorkItem), &o) : nullptr;
                if (!h) {
                    ok = false;
                    break;
                }
                std::memcpy(h, kv.second.data(), kv.second.size() * sizeof(gf::WorkItem));
                off_items.push_back(o);
            }
            if (!ok) {
                fail_worker(hipErrorOutOfMemory, "serving staging buffer too small");
                break;
            }
            for (size_t i = 0; i < fresh.size(); ++i) {
                h_args[i] = fresh[i]->args;
                h_slots[i] = fresh[i]->slot;
                h_mu2[i] = fresh[i]->p.mu2;
            }
            std::memset(h_cnt, 0, std::max<size_t>(1, groups.size()) * sizeof(unsigned));

            e = hipMemcpyAsync(st.d, st.h, st.used, hipMemcpyHostToDevice, stream);
            for (size_t k = 0; e == hipSuccess && k < uploads.size(); ++k)
                e = hipMemcpyAsync(d_arena + uploads[k].arena_off, st.d + uploads[k].stage_off,
                                   uploads[k].bytes, hipMemcpyDeviceToDevice, stream);
            if (e == hipSuccess && !fresh.empty())
                e = gf::launch_jmu_batch(d_args, reinterpret_cast<const gf::ScanArgs *>(st.d + off_args),
                                         reinterpret_cast<const int *>(st.d + off_slots),
                                         reinterpret_cast<const double *>(st.d + off_mu2),
                                         (int)fresh.size(), stream);
            if (e == hipSuccess) e = hipEventRecord(stage_ev[next_stage], stream);
            size_t gi = 0;
            for (auto &kv : groups) {
                if (e != hipSuccess) break;
                const int n = (int)kv.second.size();
                auto rit = resident.find(kv.first);
                if (rit == resident.end())
                    rit = resident
                              .emplace(kv.first, gf::serve_resident_waves(
                                                     std::get<0>(kv.first), std::get<1>(kv.first),
                                                     std::get<2>(kv.first), std::get<3>(kv.first)))
                              .first;
                const int waves = std::min(n, rit->second);
                hipStream_t cs = comp[next_comp];
                next_comp = (next_comp + 1) % kComputeStreams;
                e = hipStreamWaitEvent(cs, stage_ev[next_stage], 0);
                if (e == hipSuccess)
                    e = gf::launch_serve(d_args,
                                         reinterpret_cast<const gf::WorkItem *>(st.d + off_items[gi]),
                                         n, reinterpret_cast<unsigned *>(st.d + off_cnt) + gi,
                                         std::get<0>(kv.first), std::get<1>(kv.first),
                                         std::get<2>(kv.first), std::get<3>(kv.first), waves, cs);
                if (e == hipSuccess) e = hipEventRecord(group_ev[next_stage][gi], cs);
                if (e == hipSuccess) b.ev.push_back(group_ev[next_stage][gi]);
                ++gi;
            }
            if (e != hipSuccess) {
                fail_worker(e, "serving launch");
                break;
            }
            if (b.ev.empty()) b.ev.push_back(stage_ev[next_stage]);
            b.stage = next_stage;
            next_stage = (next_stage + 1) % kStages;
            {
                std::lock_guard<std::mutex> lock(mu);
                ++n_batches;
                n_items += b.items;
            }
            inflight.push_back(std::move(b));
        }

        // retire the oldest batch once kMaxInflight are in flight, or when
        // there was nothing new to launch
        if ((int)inflight.size() >= kMaxInflight || (!inflight.empty() && !launch_now)) {
            Batch &o = inflight.front();
            e = hipSuccess;
            for (hipEvent_t ev : o.ev)
                if (e == hipSuccess) e = hipEventSynchronize(ev);
            if (e != hipSuccess) {
                fail_worker(e, "hipEventSynchronize");
                break;
            }
            std::lock_guard<std::mutex> lock(mu);
            for (auto &rt : o.tiles) {
                Request *r = rt.first;
                r->tiles_done += rt.second;
                if (r->tiles_done == r->n_tiles) finish(r);
            }
            running.erase(std::remove_if(running.begin(), running.end(),
                                         [](Request *r) { return r->state == GF_REQ_DONE; }),
                          running.end());
            inflight.pop_front();
            cv_done.notify_all();
        }
    }
    // drain
    while (!inflight.empty()) {
        for (hipEvent_t ev : inflight.front().ev) (void)hipEventSynchronize(ev);
        inflight.pop_front();
    }
}

using gf::fail;
using gf::hip_fail;

extern "C" {

int gf_server_create(const gf_server_config *cfg, gf_server_t **out)
{
    if (!cfg || !out) return fail(GF_EINVAL, "cfg and out must not be NULL");
    *out = nullptr;
    if (cfg->device_budget_bytes < (1u << 20))
        return fail(GF_EINVAL, "device_budget_bytes must be at least 1 MiB");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 65536)
        return fail(GF_EINVAL, "max_inflight must be in [1, 65536]");
    if (!(cfg->batch_evals >= 0.0) || !std::isfinite(cfg->batch_evals))
        return fail(GF_EINVAL, "batch_evals must be finite and >= 0");
    int dev;
    int rc = gf::current_device(&dev);
    if (rc != GF_OK) return rc;
    gf_server_t *s = new (std::nothrow) gf_server_t();
    if (!s) return fail(GF_ENOMEM, "host allocation failed");
    s->device = dev;
    s->cfg = *cfg;
    if (s->cfg.batch_evals == 0.0) s->cfg.batch_evals = 4e10;
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    for (int k = 0; e == hipSuccess && k < kComputeStreams; ++k)
        e = hipStreamCreateWithFlags(&s->comp[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&s->d_arena, cfg->device_budget_bytes);
    if (e == hipSuccess) e = hipMalloc(&s->d_args, sizeof(gf::ScanArgs) * cfg->max_inflight);
    if (e == hipSuccess)
        e = hipMalloc(&s->d_jmu, 2 * sizeof(double) * (GF_MAX_TAYLOR + 1) * cfg->max_inflight);
    for (int k = 0; e == hipSuccess && k < kStages; ++k) {
        s->stage[k].bytes = kStageBytes;
        e = hipHostMalloc(reinterpret_cast<void **>(&s->stage[k].h), kStageBytes, 0);
        if (e == hipSuccess) e = hipMalloc(&s->stage[k].d, kStageBytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->stage_ev[k], hipEventDisableTiming);
        for (int g = 0; e == hipSuccess && g < kMaxGroups; ++g)
            e = hipEventCreateWithFlags(&s->group_ev[k][g], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        int r = hip_fail(e, "gf_server_create");
        gf_server_destroy(s);
        return r;
    }
    const long long waves = std::max(gf::serve_resident_waves(0, 1, 0, 0),
                                     gf::serve_resident_waves(1, 1, 0, 0));
    s->fill_min = std::min<long long>(3 * waves / 2, kMaxItemsPerBatch);
    s->fill_max = std::min<long long>(6 * waves, kMaxItemsPerBatch);
    s->arena.init(cfg->device_budget_bytes);
    for (int k = cfg->max_inflight - 1; k >= 0; --k) s->free_slots.push_back(k);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return GF_OK;
}

int gf_server_submit(gf_server_t *s, const gf_params *params, const gf_grid *grid,
                     const gf_quadrature *quad, uint64_t *ticket)
{
    return gf_server_submit_ex(s, params, nullptr, grid, quad, ticket);
}

int gf_server_submit_ex(gf_server_t *s, const gf_params *params, const gf_propagators *props,
                        const gf_grid *grid, const gf_quadrature *quad, uint64_t *ticket)
{
    if (!s || !ticket) return fail(GF_EINVAL, "NULL argument");
    int rc = gf::validate_params(params, quad);
    if (rc == GF_OK) rc = gf::validate_props(props, *quad);
    if (rc == GF_OK) rc = gf::validate_grid(*params, props, grid);
    std::lock_guard<std::mutex> lock(s->mu);
    if (rc != GF_OK) {
        ++s->n_rejected;
        return rc;
    }
    if (s->worker_error != GF_OK) return fail(s->worker_error, "%s", s->worker_msg.c_str());
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(GF_ENOMEM, "host allocation failed");
    r->p = *params;
    r->g = *grid;
    r->q = *quad;
    if (props) {
        r->props = *props;
        r->has_props = true;
    }
    r->out_bytes = (size_t)grid->n_re * (size_t)grid->n_im * 16;
    // an idle server evicts every unreferenced table, so a request is
    // admissible at some point exactly when its output and its own tables fit
    // the arena together
    const size_t need = gf::align256(r->out_bytes) + table_bytes(*quad);
    if (need > s->arena.size()) {
        delete r;
        ++s->n_rejected;
        return fail(GF_EBUDGET,
                    "request output and node tables (%zu bytes) exceed the device budget (%zu)",
                    need, s->arena.size());
    }
    r->keys[0] = key_radial(*quad, *params);
    r->keys[1] = key_angular(*quad, *params);
    r->keys[2] = key_arc(*quad);
    // one lane per point: the batch already fills the GPU with many requests,
    // and whole 64-point tiles waste no lanes on short node lists
    r->lanes = 1;
    // a numerator adds a third pair sum and three polynomials per node:
    // about 1.4 times the time per evaluation (bench box, pole sums)
    r->cost_per_tile = (64.0 / r->lanes) * nominal_evals_per_point(*quad) * (props ? props->n1 : 1) *
                       (quad->precision == GF_PREC_FP32C ? 0.6 : 1.0) *
                       (props && props->numerator ? 1.4 : 1.0);
    r->t_submit = Clock::now();
    if (!s->any_submit) {
        s->any_submit = true;
        s->first_submit = r->t_submit;
    }
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->reqs[r->ticket] = r;
    ++s->n_submitted;
    if ((long long)grid->n_re * grid->n_im == 0) {
        s->finish(r);
        s->cv_done.notify_all();
        return GF_OK;
    }
    s->pending.push_back(r);
    s->cv_work.notify_one();
    return GF_OK;
}

int gf_server_poll(gf_server_t *s, uint64_t ticket, int *state)
{
    if (!s || !state) return fail(GF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(GF_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    *state = it->second->state;
    return GF_OK;
}

int gf_server_wait(gf_server_t *s, uint64_t ticket, double timeout_ms)
{
    if (!s) return fail(GF_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lock(s->mu);
    auto done = [&] {
        auto it = s->reqs.find(ticket);
        return it == s->reqs.end() || it->second->state == GF_REQ_DONE || s->worker_error != GF_OK;
    };
    if (s->reqs.find(ticket) == s->reqs.end())
        return fail(GF_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (timeout_ms < 0) {
        s->cv_done.wait(lock, done);
    } else if (!s->cv_done.wait_for(lock, std::chrono::duration<double, std::milli>(timeout_ms),
                                    done)) {
        return 0;
    }
    if (s->worker_error != GF_OK) return fail(s->worker_error, "%s", s->worker_msg.c_str());
    return 1;
}

int gf_server_wait_any(gf_server_t *s, double timeout_ms, uint64_t *ticket)
{
    if (!s || !ticket) return fail(GF_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lock(s->mu);
    auto ready = [&] { return !s->completed.empty() || s->worker_error != GF_OK; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lock, ready);
    } else if (!s->cv_done.wait_for(lock, std::chrono::duration<double, std::milli>(timeout_ms),
                                    ready)) {
        return 0;
    }
    if (s->worker_error != GF_OK && s->completed.empty())
        return fail(s->worker_error, "%s", s->worker_msg.c_str());
    *ticket = s->completed.front();
    s->completed.pop_front();
    return 1;
}

int gf_server_result(gf_server_t *s, uint64_t ticket, const void **dev_ptr, int64_t *n_points)
{
    if (!s || !dev_ptr || !n_points) return fail(GF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(GF_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (r->state != GF_REQ_DONE) return fail(GF_EINVAL, "request %llu is not done", (unsigned long long)ticket);
    *n_points = (int64_t)r->g.n_re * r->g.n_im;
    *dev_ptr = *n_points ? s->d_arena + r->out_off : nullptr;
    return GF_OK;
}

int gf_server_copy_result(gf_server_t *s, uint64_t ticket, void *host_dst)
{
    const void *src = nullptr;
    int64_t n = 0;
    int rc = gf_server_result(s, ticket, &src, &n);
    if (rc != GF_OK) return rc;
    if (!host_dst) return fail(GF_EINVAL, "host_dst must not be NULL");
    if (n == 0) return GF_OK;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != s->device) (void)hipSetDevice(s->device);
    hipError_t e = hipMemcpy(host_dst, src, (size_t)n * 16, hipMemcpyDeviceToHost);
    if (cur != s->device && cur >= 0) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (result)");
    return GF_OK;
}

int gf_server_release(gf_server_t *s, uint64_t ticket)
{
    if (!s) return fail(GF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(GF_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (r->state != GF_REQ_DONE) return fail(GF_EINVAL, "request %llu is not done", (unsigned long long)ticket);
    if (r->slot >= 0) {
        s->arena.release(r->out_off, r->out_bytes);
        for (int k = 0; k < 3; ++k) {
            auto jt = s->tables.find(r->keys[k]);
            if (jt != s->tables.end()) --jt->second.refs;
        }
        s->free_slots.push_back(r->slot);
    }
    s->completed.erase(std::remove(s->completed.begin(), s->completed.end(), ticket),
                       s->completed.end());
    s->reqs.erase(it);
    delete r;
    ++s->n_released;
    s->admit_blocked = false;
    s->cv_work.notify_one();
    return GF_OK;
}

int gf_server_stats_get(gf_server_t *s, gf_server_stats *st)
{
    if (!s || !st) return fail(GF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = s->n_submitted;
    st->completed = s->n_completed;
    st->released = s->n_released;
    st->rejected = s->n_rejected;
    st->queued = (int64_t)s->pending.size();
    st->running = (int64_t)s->running.size();
    st->bytes_in_use = (int64_t)s->arena.used();
    st->bytes_peak = (int64_t)s->arena.peak();
    st->bytes_budget = (int64_t)s->arena.size();
    st->batches = s->n_batches;
    st->work_items = s->n_items;
    st->points_done = s->points_done;
    st->nominal_evals_done = s->nominal_evals;
    if (!s->latencies_ms.empty()) {
        std::vector<double> v = s->latencies_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            size_t i = (size_t)std::ceil(q * (double)v.size()) - 1;
            return v[std::min(i, v.size() - 1)];
        };
        double sum = 0.0;
        for (double x : v) sum += x;
        st->latency_mean_ms = sum / (double)v.size();
        st->latency_p50_ms = pct(0.50);
        st->latency_p90_ms = pct(0.90);
        st->latency_p99_ms = pct(0.99);
        st->latency_max_ms = v.back();
        st->first_submit_to_last_done_s =
            std::chrono::duration<double>(s->last_done - s->first_submit).count();
    }
    return GF_OK;
}

int gf_server_destroy(gf_server_t *s)
{
    if (!s) return GF_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (s->device >= 0 && cur != s->device) (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (int k = 0; k < kComputeStreams; ++k)
        if (s->comp[k]) (void)hipStreamSynchronize(s->comp[k]);
    for (int k = 0; k < kStages; ++k) {
        if (s->stage_ev[k]) (void)hipEventDestroy(s->stage_ev[k]);
        for (int g = 0; g < kMaxGroups; ++g)
            if (s->group_ev[k][g]) (void)hipEventDestroy(s->group_ev[k][g]);
        if (s->stage[k].h) (void)hipHostFree(s->stage[k].h);
        if (s->stage[k].d) (void)hipFree(s->stage[k].d);
    }
    if (s->d_jmu) (void)hipFree(s->d_jmu);
    if (s->d_args) (void)hipFree(s->d_args);
    if (s->d_arena) (void)hipFree(s->d_arena);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    for (int k = 0; k < kComputeStreams; ++k)
        if (s->comp[k]) (void)hipStreamDestroy(s->comp[k]);
    if (cur >= 0 && cur != s->device) (void)hipSetDevice(cur);
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
    return GF_OK;
}

}  // extern "C"
