// Continuous-batching request loop over the lbm3 C ABI (include/lbm3.h):
// a first-fit allocator over a caller-owned device pool, a FIFO queue with
// bounded overtaking, and rounds that retire finished simulations, admit
// queued ones and enqueue batched steps of everything resident.  Host code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
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

struct Request {
    uint64_t tag = 0;
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

}  // namespace

struct lbm3_server {
    char *pool = nullptr;
    size_t pool_bytes = 0;
    hipStream_t stream = nullptr;
    int max_resident = 1, max_skips = 0;
    Arena sims;                // simulation buffers: [0, sim_bytes) of the pool
    size_t sim_bytes = 0;
    char *image_dev = nullptr; // batch tables: the rest of the pool
    size_t image_cap = 0, table_used = 0;
    unsigned char *image_host = nullptr;  // pinned staging of the tables
    hipEvent_t round_done = nullptr;
    bool inflight = false;
    std::deque<Request> queue;
    std::vector<Resident> res;
    std::deque<lbm3_result> done;
    std::map<uint64_t, Kept> kept;
    std::chrono::steady_clock::time_point t0;
    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
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

lbm3_status wait_round(lbm3_server *s)
{
    if (!s->inflight) return LBM3_OK;
    s->inflight = false;
    return hipEventSynchronize(s->round_done) == hipSuccess ? LBM3_OK : LBM3_EDEVICE;
}

void retire(lbm3_server *s, size_t i, lbm3_status st)
{
    Resident &r = s->res[i];
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
    s->table_used -= r.req.table;
    s->done.push_back(o);
    s->res.erase(s->res.begin() + (long)i);
}

void admit(lbm3_server *s)
{
    for (auto it = s->queue.begin(); it != s->queue.end() && (int)s->res.size() < s->max_resident;) {
        Request &r = *it;
        size_t off = 0;
        bool fits = s->table_used + r.table + kTableSlack <= s->image_cap && s->sims.alloc(r.bytes, off);
        if (!fits) {
            // the oldest waiting request holds the line after max_skips rounds
            if (++r.skips > s->max_skips) break;
            ++it;
            continue;
        }
        Resident m;
        m.req = std::move(r);
        m.off = off;
        m.left = m.req.nsteps;
        it = s->queue.erase(it);
        lbm3_status st = lbm3_create(&m.req.p, s->pool + off, m.req.bytes, s->stream, &m.h);
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
        s->table_used += m.req.table;
        s->res.push_back(std::move(m));
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
    if (!pool || ((uintptr_t)pool & 255) != 0 || pool_bytes < (1u << 20) || max_resident < 1 || max_skips < 0)
        return LBM3_EINVAL;
    lbm3_server *s = new (std::nothrow) lbm3_server();
    if (!s) return LBM3_ENOMEM;
    s->pool = (char *)pool;
    s->pool_bytes = pool_bytes;
    s->stream = (hipStream_t)stream;
    s->max_resident = max_resident;
    s->max_skips = max_skips;
    // tables: 1/256 of the pool (at least 1 MiB) at its end
    s->image_cap = align256(std::max<size_t>(1u << 20, pool_bytes / 256));
    s->sim_bytes = (pool_bytes - s->image_cap) & ~(size_t)255;
    s->image_dev = s->pool + s->sim_bytes;
    s->sims.reset(s->sim_bytes);
    if (hipHostMalloc((void **)&s->image_host, s->image_cap, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&s->round_done, hipEventDisableTiming) != hipSuccess) {
        if (s->image_host) (void)hipHostFree(s->image_host);
        delete s;
        return LBM3_EDEVICE;
    }
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
    lbm3_derived d;
    lbm3_status st = lbm3_resolve(p, &d);
    if (st != LBM3_OK) {
        fail_result(s, r, st);
        return LBM3_OK;
    }
    // calibrated here once; the device handle gets lambda, kappa directly
    r.p.native = 1;
    for (int k = 0; k < 3; ++k) {
        r.p.lambda[k] = d.lambda[k];
        r.p.kappa[k] = d.kappa[k];
    }
    r.bytes = align256(lbm3_footprint(&r.p));
    r.table = table_share(r.p);
    if (r.bytes > s->sim_bytes || r.table + kTableSlack > s->image_cap) {
        fail_result(s, r, LBM3_ENOMEM);
        return LBM3_OK;
    }
    size_t n = (size_t)nodes_of(r.p);
    r.rho0.assign(rho0, rho0 + n);
    r.phi0.assign(phi0, phi0 + n);
    s->queue.push_back(std::move(r));
    return LBM3_OK;
}

lbm3_status lbm3_server_run(lbm3_server *s, int64_t quantum, int32_t *n_resident, int32_t *n_queued)
{
    if (!s || quantum < 1) return LBM3_EINVAL;
    lbm3_status st = wait_round(s);
    if (st != LBM3_OK) return st;
    for (size_t i = s->res.size(); i-- > 0;)
        if (s->res[i].left == 0) retire(s, i, LBM3_OK);
    admit(s);
    if (!s->res.empty()) {
        // most steps left first: each later segment is a prefix of this order
        std::stable_sort(s->res.begin(), s->res.end(),
                         [](const Resident &a, const Resident &b) { return a.left > b.left; });
        std::vector<lbm3 *> hs(s->res.size());
        for (size_t i = 0; i < hs.size(); ++i) hs[i] = s->res[i].h;
        lbm3b::Image img;
        st = lbm3b::build(hs.data(), (int)hs.size(), img);
        if (st != LBM3_OK) return st;
        if (img.bytes.size() > s->image_cap) return LBM3_ENOMEM;
        std::memcpy(s->image_host, img.bytes.data(), img.bytes.size());
        if (hipMemcpyAsync(s->image_dev, s->image_host, img.bytes.size(), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess)
            return LBM3_EDEVICE;
        int64_t prev = 0;
        for (size_t k = hs.size(); k-- > 0;) {
            int64_t a = std::min<int64_t>(quantum, s->res[k].left);
            if (a > prev) {
                st = lbm3b::enqueue(hs.data(), (int)k + 1, img, s->image_dev, prev, a - prev, s->stream);
                if (st != LBM3_OK) return st;
                prev = a;
            }
        }
        for (auto &r : s->res) r.left -= std::min<int64_t>(quantum, r.left);
        if (hipEventRecord(s->round_done, s->stream) != hipSuccess) return LBM3_EDEVICE;
        s->inflight = true;
    }
    if (n_resident) *n_resident = (int32_t)s->res.size();
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
    lbm3_status st = wait_round(s);
    for (auto &r : s->res) lbm3_destroy(r.h);
    if (s->image_host) (void)hipHostFree(s->image_host);
    if (s->round_done) (void)hipEventDestroy(s->round_done);
    delete s;
    return st;
}

}  // extern "C"
