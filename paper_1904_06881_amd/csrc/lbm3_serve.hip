// Continuous-batching request loop over the lbm3 C ABI (include/lbm3.h):
// a first-fit allocator over a caller-owned device pool, a FIFO queue with
// bounded overtaking, and rounds that retire finished simulations, admit
// queued ones and enqueue batched steps of everything resident.  Host code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/lbm3.h"
#include "lbm3_batch.h"

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// room kept in the table area for per-launch alignment
const size_t kTableSlack = 64u << 10;

// first-fit allocator over [0, size) with coalescing frees
struct Arena {
    std::map<size_t, size_t> free_;  // offset -> length
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t len, size_t &off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            off = it->first;
            size_t rest = it->second - len;
            free_.erase(it);
            if (rest) free_[off + len] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t len)
    {
        auto it = free_.emplace(off, len).first;
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
};

// Calibration of a request's (lambda, kappa) from its tensions and width
// (lbm3_resolve, host only) runs on worker threads while the GPU steps the
// resident simulations; a request is admitted once its calibration is done.
struct Calib {
    std::atomic<int> state{0};  // 0 pending, 1 done
    lbm3_params p{};
    lbm3_status st = LBM3_OK;
    lbm3_derived d{};
};

struct CalibPool {
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Calib>> jobs;
    bool stop = false;
    void start(int n)
    {
        for (int i = 0; i < n; ++i)
            workers.emplace_back([this] {
                for (;;) {
                    std::shared_ptr<Calib> c;
                    {
                        std::unique_lock<std::mutex> lk(mu);
                        cv.wait(lk, [this] { return stop || !jobs.empty(); });
                        if (stop && jobs.empty()) return;
                        c = jobs.front();
                        jobs.pop_front();
                    }
                    c->st = lbm3_resolve(&c->p, &c->d);
                    c->state.store(1, std::memory_order_release);
                }
            });
    }
    void push(std::shared_ptr<Calib> c)
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            jobs.push_back(std::move(c));
        }
        cv.notify_one();
    }
    void finish()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        for (auto &t : workers) t.join();
        workers.clear();
    }
};

struct Request {
    uint64_t tag = 0;
    std::shared_ptr<Calib> calib;  // null once applied to p
    lbm3_params p{};
    std::vector<double> rho0, phi0;
    int64_t nsteps = 0;
    uint32_t flags = 0;
    double t_submit = 0;
    int skips = 0;
    size_t bytes = 0, table = 0;
};

struct Resident {
    Request req;
    lbm3 *h = nullptr;
    size_t off = 0;
    int64_t left = 0;
    double t_admit = 0;
};

struct Kept {
    std::vector<double> rho, phi;
};

int64_t nodes_of(const lbm3_params &p)
{
    return (int64_t)p.n[0] * p.n[1] * (p.lattice == LBM3_D3Q27 ? p.n[2] : 1);
}

// bytes of the batch tables one simulation adds: its descriptor and one int
// per block of its moments, ghost-layer and fused launches (bounded above)
size_t table_share(const lbm3_params &p)
{
    int64_t N = nodes_of(p);
    int64_t per_plane = p.lattice == LBM3_D3Q27 ? (int64_t)p.n[0] * p.n[1] : p.n[0];
    int64_t blocks = N / 256 + 1;            // moments
    blocks += 2 * per_plane / 256 + 1;       // ghost layers
    blocks += N / (62 * 2) + per_plane + 64;  // fused: at least 2 planes of >= 62 nodes per block
    return align256(1024 + 4 * (size_t)blocks);
}

// Simulations are split by size into lanes, each with its own stream, batch
// tables and round cadence, so that small grids are not held to the step
// time of large ones; lanes run concurrently on the GPU.
const int kLanes = 2;
const int64_t kSmallNodes = 1 << 18;  // lane 0 below, lane 1 from here on

int lane_of(const lbm3_params &p) { return nodes_of(p) < kSmallNodes ? 0 : 1; }
// large lane: at most this many nodes resident together (a single grid of
// any size is always admitted).  Grids this large fill the GPU alone, so
// running more of them at once only slows each: on the bench's request
// stream, without the limit the largest requests finished 19 % later than
// one at a time (p99 2.37 s against 1.99 s); with it p99 matched (2.00 s)
// and the median fell from 0.11 s to 0.06 s (small grids get more of the GPU).
const int64_t kLargeLaneNodes = 1LL << 23;

struct Lane {
    hipStream_t stream = nullptr;
    char *image_dev = nullptr;            // batch tables of this lane in the pool
    unsigned char *image_host = nullptr;  // pinned staging of the tables
    size_t image_cap = 0, table_used = 0;
    hipEvent_t round_done = nullptr;
    bool inflight = false;
    std::vector<Resident> res;
};

}  // namespace

struct lbm3_server {
    char *pool = nullptr;
    size_t pool_bytes = 0;
    int max_resident = 1, max_skips = 0;
    Arena sims;                // simulation buffers: [0, sim_bytes) of the pool
    size_t sim_bytes = 0;
    Lane lane[kLanes];
    std::deque<Request> queue;
    CalibPool calib;
    std::deque<lbm3_result> done;
    std::map<uint64_t, Kept> kept;
    std::chrono::steady_clock::time_point t0;
    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    int resident() const
    {
        int n = 0;
        for (const auto &l : lane) n += (int)l.res.size();
        return n;
    }
};

namespace {

void fail_result(lbm3_server *s, const Request &r, lbm3_status st)
{
    lbm3_result o{};
    o.tag = r.tag;
    o.status = st;
    o.nodes = nodes_of(r.p);
    o.t_submit = o.t_admit = o.t_done = r.t_submit;
    s->done.push_back(o);
}

// 1: the lane's last round is done (or none is in flight), 0: still running
int lane_ready(Lane &l, bool block, lbm3_status &st)
{
    st = LBM3_OK;
    if (!l.inflight) return 1;
    hipError_t e = block ? hipEventSynchronize(l.round_done) : hipEventQuery(l.round_done);
    if (e == hipErrorNotReady) return 0;
    l.inflight = false;
    if (e != hipSuccess) st = LBM3_EDEVICE;
    return 1;
}

void retire(lbm3_server *s, Lane &l, size_t i, lbm3_status st)
{
    Resident &r = l.res[i];
    lbm3_result o{};
    o.tag = r.req.tag;
    o.nodes = nodes_of(r.req.p);
    o.t_submit = r.req.t_submit;
    o.t_admit = r.t_admit;
    o.bytes = (double)(r.req.bytes + r.req.table);
    o.status = st;
    if (st == LBM3_OK) {
        int q = lbm3_observe(r.h, LBM3_OBS_SUMS, &o.obs, nullptr, nullptr, nullptr, nullptr);
        if (q != LBM3_OK) o.status = q;  // LBM3_EUNSTABLE: non-finite or non-positive fields
        o.steps = o.obs.step;
        if ((r.req.flags & LBM3_SERVE_FIELDS) && o.status == LBM3_OK) {
            Kept k;
            k.rho.resize(o.nodes);
            k.phi.resize(o.nodes);
            if (lbm3_observe(r.h, LBM3_OBS_FIELDS, nullptr, k.rho.data(), k.phi.data(), nullptr, nullptr) ==
                LBM3_OK) {
                s->kept[o.tag] = std::move(k);
                o.has_fields = 1;
            }
        }
    }
    o.t_done = s->now();
    lbm3_destroy(r.h);
    s->sims.release(r.off, r.req.bytes);
    l.table_used -= r.req.table;
    s->done.push_back(o);
    l.res.erase(l.res.begin() + (long)i);
}

// admit queued requests of lane li in arrival order while they fit
void admit(lbm3_server *s, int li)
{
    Lane &l = s->lane[li];
    for (auto it = s->queue.begin(); it != s->queue.end() && s->resident() < s->max_resident;) {
        Request &r = *it;
        if (lane_of(r.p) != li) {
            ++it;
            continue;
        }
        if (r.calib) {
            // still calibrating: later requests may go first (not counted as a skip)
            if (r.calib->state.load(std::memory_order_acquire) == 0) {
                ++it;
                continue;
            }
            if (r.calib->st != LBM3_OK) {
                fail_result(s, r, r.calib->st);
                it = s->queue.erase(it);
                continue;
            }
            r.p.native = 1;
            for (int k = 0; k < 3; ++k) {
                r.p.lambda[k] = r.calib->d.lambda[k];
                r.p.kappa[k] = r.calib->d.kappa[k];
            }
            r.calib.reset();
        }
        size_t off = 0;
        int64_t lane_nodes = 0;
        for (const Resident &m : l.res) lane_nodes += nodes_of(m.req.p);
        const bool room = li == 0 || l.res.empty() || lane_nodes + nodes_of(r.p) <= kLargeLaneNodes;
        bool fits = room && l.table_used + r.table + kTableSlack <= l.image_cap && s->sims.alloc(r.bytes, off);
        if (!fits) {
            // the oldest waiting request holds its lane after max_skips rounds
            if (++r.skips > s->max_skips) break;
            ++it;
            continue;
        }
        Resident m;
        m.req = std::move(r);
        m.off = off;
        m.left = m.req.nsteps;
        it = s->queue.erase(it);
        lbm3_status st = lbm3_create(&m.req.p, s->pool + off, m.req.bytes, l.stream, &m.h);
        if (st == LBM3_OK) st = lbm3_init(m.h, m.req.rho0.data(), m.req.phi0.data());
        if (st != LBM3_OK) {
            if (m.h) lbm3_destroy(m.h);
            s->sims.release(off, m.req.bytes);
            fail_result(s, m.req, st);
            continue;
        }
        m.t_admit = s->now();
        m.req.rho0 = std::vector<double>();
        m.req.phi0 = std::vector<double>();
        l.table_used += m.req.table;
        l.res.push_back(std::move(m));
    }
}

// enqueue up to `quantum` batched steps of every resident of the lane
lbm3_status enqueue_round(Lane &l, int64_t quantum)
{
    if (l.res.empty()) return LBM3_OK;
    // most steps left first: each later segment is a prefix of this order
    std::stable_sort(l.res.begin(), l.res.end(), [](const Resident &a, const Resident &b) { return a.left > b.left; });
    std::vector<lbm3 *> hs(l.res.size());
    for (size_t i = 0; i < hs.size(); ++i) hs[i] = l.res[i].h;
    lbm3b::Image img;
    lbm3_status st = lbm3b::build(hs.data(), (int)hs.size(), img);
    if (st != LBM3_OK) return st;
    if (img.bytes.size() > l.image_cap) return LBM3_ENOMEM;
    std::memcpy(l.image_host, img.bytes.data(), img.bytes.size());
    if (hipMemcpyAsync(l.image_dev, l.image_host, img.bytes.size(), hipMemcpyHostToDevice, l.stream) != hipSuccess)
        return LBM3_EDEVICE;
    int64_t prev = 0;
    for (size_t k = hs.size(); k-- > 0;) {
        int64_t a = std::min<int64_t>(quantum, l.res[k].left);
        if (a > prev) {
            st = lbm3b::enqueue(hs.data(), (int)k + 1, img, l.image_dev, prev, a - prev, l.stream);
            if (st != LBM3_OK) return st;
            prev = a;
        }
    }
    for (auto &r : l.res) r.left -= std::min<int64_t>(quantum, r.left);
    if (hipEventRecord(l.round_done, l.stream) != hipSuccess) return LBM3_EDEVICE;
    l.inflight = true;
    return LBM3_OK;
}

void release_lanes(lbm3_server *s)
{
    for (auto &l : s->lane) {
        if (l.image_host) (void)hipHostFree(l.image_host);
        if (l.round_done) (void)hipEventDestroy(l.round_done);
        if (l.stream) (void)hipStreamDestroy(l.stream);
    }
}

}  // namespace

extern "C" {

size_t lbm3_server_request_bytes(const lbm3_params *p)
{
    size_t f = lbm3_footprint(p);
    return f ? align256(f) + table_share(*p) : 0;
}

lbm3_status lbm3_server_create(void *pool, size_t pool_bytes, void *stream, int32_t max_resident,
                               int32_t max_skips, lbm3_server **out)
{
    if (!out) return LBM3_EINVAL;
    *out = nullptr;
    if (!pool || ((uintptr_t)pool & 255) != 0 || pool_bytes < (4u << 20) || max_resident < 1 || max_skips < 0)
        return LBM3_EINVAL;
    lbm3_server *s = new (std::nothrow) lbm3_server();
    if (!s) return LBM3_ENOMEM;
    s->pool = (char *)pool;
    s->pool_bytes = pool_bytes;
    s->max_resident = max_resident;
    s->max_skips = max_skips;
    // tables: 1/256 of the pool (at least 1 MiB) per lane at its end
    size_t cap = align256(std::max<size_t>(1u << 20, pool_bytes / 256));
    s->sim_bytes = (pool_bytes - kLanes * cap) & ~(size_t)255;
    s->sims.reset(s->sim_bytes);
    // lane streams start after the work already on the caller's stream
    hipEvent_t ready = nullptr;
    bool ok = hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess &&
              hipEventRecord(ready, (hipStream_t)stream) == hipSuccess;
    for (int i = 0; i < kLanes && ok; ++i) {
        Lane &l = s->lane[i];
        l.image_cap = cap;
        l.image_dev = s->pool + s->sim_bytes + (size_t)i * cap;
        ok = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) == hipSuccess &&
             hipHostMalloc((void **)&l.image_host, cap, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&l.round_done, hipEventDisableTiming) == hipSuccess &&
             hipStreamWaitEvent(l.stream, ready, 0) == hipSuccess;
    }
    if (ready) (void)hipEventDestroy(ready);
    if (!ok) {
        release_lanes(s);
        delete s;
        return LBM3_EDEVICE;
    }
    s->calib.start((int)std::max(1u, std::min(8u, std::thread::hardware_concurrency())));
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return LBM3_OK;
}

lbm3_status lbm3_server_submit(lbm3_server *s, const lbm3_params *p, const double *rho0, const double *phi0,
                               int64_t nsteps, uint64_t tag, uint32_t flags)
{
    if (!s || !p || !rho0 || !phi0 || nsteps < 0) return LBM3_EINVAL;
    Request r;
    r.tag = tag;
    r.p = *p;
    r.nsteps = nsteps;
    r.flags = flags;
    r.t_submit = s->now();
    // the footprint does not depend on lambda, kappa: checked here, the
    // calibration itself runs on a worker thread (applied at admission)
    const size_t fp = lbm3_footprint(&r.p);
    if (!fp) {
        fail_result(s, r, LBM3_EINVAL);
        return LBM3_OK;
    }
    r.bytes = align256(fp);
    r.table = table_share(r.p);
    if (r.bytes > s->sim_bytes || r.table + kTableSlack > s->lane[lane_of(r.p)].image_cap) {
        fail_result(s, r, LBM3_ENOMEM);
        return LBM3_OK;
    }
    size_t n = (size_t)nodes_of(r.p);
    r.rho0.assign(rho0, rho0 + n);
    r.phi0.assign(phi0, phi0 + n);
    if (!r.p.native) {
        r.calib = std::make_shared<Calib>();
        r.calib->p = r.p;
        s->calib.push(r.calib);
    }
    s->queue.push_back(std::move(r));
    return LBM3_OK;
}

lbm3_status lbm3_server_run(lbm3_server *s, int64_t quantum, int32_t *n_resident, int32_t *n_queued)
{
    if (!s || quantum < 1) return LBM3_EINVAL;
    // serve every lane whose last round is done; return once a lane has
    // enqueued work or produced results, or when nothing is on the GPU
    for (;;) {
        bool busy = false, acted = false;
        for (int i = 0; i < kLanes; ++i) {
            Lane &l = s->lane[i];
            lbm3_status st;
            if (!lane_ready(l, false, st)) {
                busy = true;
                continue;
            }
            if (st != LBM3_OK) return st;
            const size_t results = s->done.size();
            for (size_t k = l.res.size(); k-- > 0;)
                if (l.res[k].left == 0) retire(s, l, k, LBM3_OK);
            admit(s, i);
            if ((st = enqueue_round(l, quantum)) != LBM3_OK) return st;
            acted = acted || l.inflight || s->done.size() != results;
        }
        // nothing to do yet but a queued request is still calibrating: wait for it
        if (!acted && !busy)
            for (const Request &r : s->queue)
                if (r.calib && r.calib->state.load(std::memory_order_acquire) == 0) {
                    busy = true;
                    break;
                }
        if (acted || !busy) break;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    if (n_resident) *n_resident = (int32_t)s->resident();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return LBM3_OK;
}

int32_t lbm3_server_poll(lbm3_server *s, lbm3_result *out)
{
    if (!s || !out) return LBM3_EINVAL;
    if (s->done.empty()) return 0;
    *out = s->done.front();
    s->done.pop_front();
    return 1;
}

lbm3_status lbm3_server_fields(lbm3_server *s, uint64_t tag, double *rho_out, double *phi_out)
{
    if (!s) return LBM3_EINVAL;
    auto it = s->kept.find(tag);
    if (it == s->kept.end()) return LBM3_EINVAL;
    if (rho_out) std::memcpy(rho_out, it->second.rho.data(), it->second.rho.size() * sizeof(double));
    if (phi_out) std::memcpy(phi_out, it->second.phi.data(), it->second.phi.size() * sizeof(double));
    s->kept.erase(it);
    return LBM3_OK;
}

double lbm3_server_clock(const lbm3_server *s) { return s ? s->now() : 0.0; }

lbm3_status lbm3_server_destroy(lbm3_server *s)
{
    if (!s) return LBM3_EINVAL;
    lbm3_status st = LBM3_OK;
    for (auto &l : s->lane) {
        lbm3_status q;
        lane_ready(l, true, q);
        if (q != LBM3_OK) st = q;
        for (auto &r : l.res) lbm3_destroy(r.h);
    }
    s->calib.finish();
    release_lanes(s);
    delete s;
    return st;
}

}  // extern "C"
