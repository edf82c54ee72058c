// Request server: a queue of Fock-build requests for many cells, admitted by
// device-memory footprint into one arena and run on worker threads, each
// build on its own HIP stream so that builds of different cells overlap on
// the device.  The contract is documented with the C declarations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "handle.h"
#include "pbcjk.h"

using namespace pbcjk;
using Clock = std::chrono::steady_clock;

namespace {

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

template <class T>
void append_bytes(std::string &s, const T *p, size_t n)
{
    s.append((const char *)p, n * sizeof(T));
}

// Deep copy of one cell's inputs; `sig` is their byte image (cache identity).
struct CellInputs {
    pbc_cell cell{};
    int natom = 0, nshell = 0;
    std::vector<double> xyz, charge, exps, coefs;
    std::vector<int> atom, l, pure, nprim;
    double omega = 0.0;
    bool has_thr = false;
    pbc_jk_thresholds thr{};
    std::string sig;

    pbc_atoms atoms() const { return pbc_atoms{natom, xyz.data(), charge.empty() ? nullptr : charge.data()}; }
    pbc_basis basis() const
    {
        return pbc_basis{nshell, atom.data(), l.data(), pure.data(), nprim.data(), exps.data(), coefs.data()};
    }
};

int copy_inputs(const pbc_cell *cell, const pbc_atoms *atoms, const pbc_basis *basis, double omega,
                const pbc_jk_thresholds *thr, CellInputs &c, std::string &err)
{
    if (!cell || !atoms || !basis) { err = "cell, atoms and basis are required"; return PBC_JK_EINVAL; }
    if (atoms->natom <= 0 || !atoms->xyz) { err = "atoms: natom > 0 and xyz are required"; return PBC_JK_EINVAL; }
    if (basis->nshell <= 0 || !basis->atom || !basis->l || !basis->pure || !basis->nprim || !basis->exps ||
        !basis->coefs) {
        err = "basis: nshell > 0 and all arrays are required";
        return PBC_JK_EINVAL;
    }
    long np = 0;
    for (int s = 0; s < basis->nshell; ++s) {
        if (basis->nprim[s] <= 0) { err = "basis: nprim must be positive"; return PBC_JK_EINVAL; }
        np += basis->nprim[s];
    }
    c.cell = *cell;
    c.natom = atoms->natom;
    c.nshell = basis->nshell;
    c.xyz.assign(atoms->xyz, atoms->xyz + 3 * (size_t)c.natom);
    if (atoms->charge) c.charge.assign(atoms->charge, atoms->charge + c.natom);
    c.atom.assign(basis->atom, basis->atom + c.nshell);
    c.l.assign(basis->l, basis->l + c.nshell);
    c.pure.assign(basis->pure, basis->pure + c.nshell);
    c.nprim.assign(basis->nprim, basis->nprim + c.nshell);
    c.exps.assign(basis->exps, basis->exps + np);
    c.coefs.assign(basis->coefs, basis->coefs + np);
    c.omega = omega;
    c.has_thr = thr != nullptr;
    if (thr) c.thr = *thr;
    c.sig.clear();
    append_bytes(c.sig, c.cell.a, 9);
    append_bytes(c.sig, &c.natom, 1);
    append_bytes(c.sig, c.xyz.data(), c.xyz.size());
    append_bytes(c.sig, &c.nshell, 1);
    append_bytes(c.sig, c.atom.data(), c.atom.size());
    append_bytes(c.sig, c.l.data(), c.l.size());
    append_bytes(c.sig, c.pure.data(), c.pure.size());
    append_bytes(c.sig, c.nprim.data(), c.nprim.size());
    append_bytes(c.sig, c.exps.data(), c.exps.size());
    append_bytes(c.sig, c.coefs.data(), c.coefs.size());
    append_bytes(c.sig, &c.omega, 1);
    const double th[8] = {c.thr.pair_R, c.thr.pair_cs, c.thr.ewald_R, c.thr.ewald_K,
                          c.thr.schwarz, c.thr.fp32_below, c.thr.r_cut, c.thr.g_cut};
    const int ht = c.has_thr ? 1 : 0;
    append_bytes(c.sig, &ht, 1);
    append_bytes(c.sig, th, 8);
    return 0;
}

// A cell known to the server.  h == nullptr while its setup is being made:
// it is then a placeholder that belongs to the request `owner` (requests for
// the same cell with other densities share the entry and wait for it).
struct Cell {
    pbc_jk *h = nullptr;
    unsigned long long owner = 0;
    bool busy = false;
    unsigned long long last_use = 0;
    size_t bytes = 0;
};

enum class RState { Queued, Working, Building, Done };

struct Request {
    unsigned long long id = 0;
    CellInputs in;
    std::vector<double> D;
    double *J = nullptr, *K = nullptr, *E_J = nullptr, *E_K = nullptr;
    RState state = RState::Queued;
    bool cancel = false;
    int status = 0;
    std::string err;
    Clock::time_point t_submit, t_start, t_done;
    bool started = false;
    double setup_ms = 0.0, build_ms = 0.0;
    int cache_hit = 0, retries = 0, nbf = 0;
    size_t dev_bytes = 0;
    pbc_jk *prepared = nullptr;  // host setup done, device part not yet created
    size_t fixed = 0, need = 0;  // device bytes: without / with the neighbour lists
    double key = 0.0;            // queue order (ascending)
};

// Estimated build seconds per squared AO: about 16 s for the largest serving
// cells (nbf ~ 1500) and 0.6 s at nbf ~ 300 on one MI355X.
constexpr double kBuildSecPerNbf2 = 6.8e-6;

}  // namespace

struct pbc_jk_server {
    pbc_jk_server_config cfg{};
    int device = 0;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;  // ascending key
    Clock::time_point t0 = Clock::now();
    std::unordered_map<unsigned long long, Request *> reqs;
    std::unordered_map<std::string, Cell *> cells;
    std::vector<std::thread> workers;
    bool stopping = false;
    unsigned long long next_id = 1, tick = 0;
    size_t reserved = 0;
    int running = 0;
    pbc_jk_server_counters c{};
};

namespace {

size_t available(pbc_jk_server *s)
{
    const size_t used = s->arena.in_use() + s->reserved;
    return used >= s->arena.capacity() ? 0 : s->arena.capacity() - used;
}

// Completes a request (lock held).
void finish(pbc_jk_server *s, Request *r, int status, const std::string &msg)
{
    r->status = status;
    r->err = msg;
    r->state = RState::Done;
    r->t_done = Clock::now();
    if (status == 0) s->c.completed++;
    else if (status == PBC_JK_ECANCELED) s->c.cancelled++;
    else s->c.failed++;
    s->cv_done.notify_all();
}

// Drops the placeholder cell that request r created, if it still holds one
// (a placeholder of another request for the same cell is left alone), and
// returns r's prepared handle for deletion outside the lock (lock held).
pbc_jk *drop_placeholder(pbc_jk_server *s, Request *r)
{
    auto it = s->cells.find(r->in.sig);
    if (it != s->cells.end() && it->second->h == nullptr && it->second->owner == r->id) {
        delete it->second;
        s->cells.erase(it);
    }
    pbc_jk *h = r->prepared;
    r->prepared = nullptr;
    return h;
}

// Inserts by key (ties by id), so the queue stays in the policy's order.
void enqueue(pbc_jk_server *s, Request *r)
{
    auto it = std::lower_bound(s->queue.begin(), s->queue.end(), r, [](const Request *a, const Request *b) {
        return a->key < b->key || (a->key == b->key && a->id < b->id);
    });
    s->queue.insert(it, r);
}

void requeue(pbc_jk_server *s, Request *r)
{
    r->state = RState::Queued;
    enqueue(s, r);
}

// Evicts idle resident cells, least recently used first, until `need` bytes
// will be available once the evicted handles are deleted, or none is left
// (lock held).  Returns the handles to delete outside the lock.  New cells
// are admitted in arrival order, so the bytes freed go to the request that
// asked for them.
std::vector<pbc_jk *> evict_for(pbc_jk_server *s, size_t need)
{
    std::vector<pbc_jk *> out;
    size_t pending = 0;
    while (available(s) + pending < need) {
        auto best = s->cells.end();
        for (auto it = s->cells.begin(); it != s->cells.end(); ++it)
            if (!it->second->busy && it->second->h &&
                (best == s->cells.end() || it->second->last_use < best->second->last_use))
                best = it;
        if (best == s->cells.end()) break;
        out.push_back(best->second->h);
        pending += best->second->bytes;
        delete best->second;
        s->cells.erase(best);
        s->c.evictions++;
    }
    return out;
}

enum Action { kNone = 0, kRunResident = 1, kPrepare = 2, kCreate = 3 };

// Chooses the next piece of work (lock held).
Action pick(pbc_jk_server *s, Request *&r, Cell *&cell, std::vector<pbc_jk *> &to_delete)
{
    bool mem_blocked = false;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request *q = *it;
        if (q->cancel) {
            if (pbc_jk *h = drop_placeholder(s, q)) to_delete.push_back(h);
            it = s->queue.erase(it);
            finish(s, q, PBC_JK_ECANCELED, "cancelled");
            continue;
        }
        auto ce = s->cells.find(q->in.sig);
        const bool own_placeholder =
            q->prepared && ce != s->cells.end() && ce->second->h == nullptr && ce->second->owner == q->id;
        if (ce != s->cells.end() && !own_placeholder) {
            if (ce->second->busy) { ++it; continue; }
            ce->second->busy = true;
            cell = ce->second;
            r = q;
            s->queue.erase(it);
            return kRunResident;
        }
        if (mem_blocked) { ++it; continue; }
        if (!q->prepared) {
            cell = new Cell();
            cell->busy = true;
            cell->owner = q->id;
            s->cells[q->in.sig] = cell;
            r = q;
            s->queue.erase(it);
            return kPrepare;
        }
        if (q->need > available(s)) {
            auto ev = evict_for(s, q->need);
            to_delete.insert(to_delete.end(), ev.begin(), ev.end());
        }
        if (q->need <= available(s)) {
            s->reserved += q->need;
            cell = ce->second;
            r = q;
            s->queue.erase(it);
            return kCreate;
        }
        mem_blocked = true;
        ++it;
    }
    return kNone;
}

void worker(pbc_jk_server *s)
{
    (void)hipSetDevice(s->device);
    std::vector<pbc_jk *> to_delete;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        Request *r = nullptr;
        Cell *cell = nullptr;
        Action act = kNone;
        s->cv_work.wait(lk, [&] {
            if (s->stopping) return true;
            act = pick(s, r, cell, to_delete);
            return act != kNone || !to_delete.empty();
        });
        if (!to_delete.empty()) {
            // evictions may have been made for work picked in this pass
            lk.unlock();
            std::vector<pbc_jk *> hs;
            hs.swap(to_delete);
            for (pbc_jk *h : hs) handle_delete(h);
            lk.lock();
            s->cv_work.notify_all();
        }
        if (act == kNone) {
            if (s->stopping) return;
            continue;
        }
        r->state = RState::Working;
        if (!r->started) {
            r->started = true;
            r->t_start = Clock::now();
        }
        s->running++;
        s->c.peak_running = std::max(s->c.peak_running, s->running);

        if (act == kPrepare) {
            lk.unlock();
            const auto t0 = Clock::now();
            const pbc_atoms at = r->in.atoms();
            const pbc_basis bs = r->in.basis();
            pbc_jk *h = nullptr;
            int rc = handle_new(&r->in.cell, &at, &bs, r->in.omega, r->in.has_thr ? &r->in.thr : nullptr, &h);
            std::string msg = rc ? pbc_jk_last_error() : "";
            size_t fixed = 0;
            if (!rc) fixed = handle_fixed_bytes(h, s->cfg.lr_budget_mb);
            r->setup_ms += ms_between(t0, Clock::now());
            lk.lock();
            s->running--;
            if (rc) {
                drop_placeholder(s, r);
                finish(s, r, rc, msg);
            } else {
                r->prepared = h;
                r->fixed = r->need = fixed;
                if (fixed > s->arena.capacity()) {
                    to_delete.push_back(drop_placeholder(s, r));
                    finish(s, r, PBC_JK_ENOMEM, "the cell's device footprint exceeds the server's HBM budget");
                } else {
                    requeue(s, r);
                }
            }
            s->cv_work.notify_all();
            continue;
        }

        if (act == kCreate) {
            pbc_jk *h = r->prepared;
            const size_t need = r->need;
            lk.unlock();
            const auto t0 = Clock::now();
            int rc = handle_device(h, &s->arena, false, s->cfg.lr_budget_mb);
            std::string msg = rc ? pbc_jk_last_error() : "";
            const size_t nbr = handle_nbr_bytes(h);
            r->setup_ms += ms_between(t0, Clock::now());
            lk.lock();
            s->reserved -= std::min(s->reserved, need);
            if (rc == PBC_JK_ENOMEM) {
                // the budget was short (neighbour lists larger than reserved,
                // or fragmentation): wait for memory with the exact footprint
                s->running--;
                r->retries++;
                s->c.retries++;
                if (nbr) r->need = r->fixed + nbr;
                if (r->need > s->arena.capacity()) {
                    to_delete.push_back(drop_placeholder(s, r));
                    finish(s, r, PBC_JK_ENOMEM, "the cell's device footprint exceeds the server's HBM budget");
                } else {
                    requeue(s, r);
                }
                s->cv_work.notify_all();
                continue;
            }
            if (rc) {
                s->running--;
                to_delete.push_back(drop_placeholder(s, r));
                finish(s, r, rc, msg);
                s->cv_work.notify_all();
                continue;
            }
            cell->h = h;
            cell->bytes = handle_dev_bytes(h);
            r->prepared = nullptr;
        } else {
            r->cache_hit = 1;
            s->c.cache_hits++;
            // repeated builds of a resident cell replay its captured graph
            if (s->cfg.use_graphs) (void)pbc_jk_set_graph(cell->h, 1);
        }

        // build on the cell (busy, resident)
        if (r->cancel) {
            cell->busy = false;
            s->running--;
            finish(s, r, PBC_JK_ECANCELED, "cancelled");
            s->cv_work.notify_all();
            continue;
        }
        r->state = RState::Building;
        pbc_jk *h = cell->h;
        lk.unlock();
        const auto t0 = Clock::now();
        int rc = pbc_jk_build(h, r->D.data(), r->J, r->K, r->E_J, r->E_K);
        std::string msg = rc ? pbc_jk_last_error() : "";
        r->build_ms = ms_between(t0, Clock::now());
        r->nbf = pbc_jk_nbf(h);
        r->dev_bytes = handle_dev_bytes(h);
        lk.lock();
        s->running--;
        cell->busy = false;
        cell->last_use = ++s->tick;
        if (!s->cfg.cache_cells || rc == PBC_JK_EDEVICE) {
            s->cells.erase(r->in.sig);
            pbc_jk *drop = cell->h;
            delete cell;
            // the cell's memory goes back to the arena before the request
            // completes, so that a completed request holds no arena bytes
            lk.unlock();
            handle_delete(drop);
            lk.lock();
        }
        finish(s, r, rc, msg);
        s->cv_work.notify_all();
        if (!to_delete.empty()) {
            lk.unlock();
            std::vector<pbc_jk *> hs;
            hs.swap(to_delete);
            for (pbc_jk *x : hs) handle_delete(x);
            lk.lock();
            s->cv_work.notify_all();
        }
    }
}

}  // namespace

extern "C" {

int pbc_jk_server_create(const pbc_jk_server_config *cfg, pbc_jk_server **out)
{
    if (!out) return PBC_JK_EINVAL;
    *out = nullptr;
    pbc_jk_server *s = new (std::nothrow) pbc_jk_server();
    if (!s) return PBC_JK_ENOMEM;
    if (cfg) s->cfg = *cfg;
    if (s->cfg.slots <= 0) s->cfg.slots = 4;
    if (s->cfg.policy != PBC_JK_SERVE_ARRIVAL && s->cfg.policy != PBC_JK_SERVE_DEADLINE) {
        delete s;
        return PBC_JK_EINVAL;
    }
    if (s->cfg.slots > 64) {
        delete s;
        return PBC_JK_EINVAL;
    }
    if (!(s->cfg.lr_budget_mb > 0.0)) s->cfg.lr_budget_mb = 1024.0;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return PBC_JK_EDEVICE;
    }
    size_t budget = s->cfg.hbm_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return PBC_JK_EDEVICE;
        }
        budget = fr / 2;
    }
    if (s->arena.init(budget) != hipSuccess) {
        delete s;
        return PBC_JK_ENOMEM;
    }
    s->c.slots = s->cfg.slots;
    s->c.budget = s->arena.capacity();
    try {
        for (int i = 0; i < s->cfg.slots; ++i) s->workers.emplace_back(worker, s);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stopping = true;
        }
        s->cv_work.notify_all();
        for (auto &t : s->workers) t.join();
        delete s;
        return PBC_JK_ENOMEM;
    }
    *out = s;
    return 0;
}

int pbc_jk_server_submit(pbc_jk_server *s, const pbc_cell *cell, const pbc_atoms *atoms, const pbc_basis *basis,
                         double omega, const pbc_jk_thresholds *thr, const double *D, double *J, double *K,
                         double *E_J, double *E_K, unsigned long long *ticket)
{
    if (!s || !ticket || !D) return PBC_JK_EINVAL;
    Request *r = new (std::nothrow) Request();
    if (!r) return PBC_JK_ENOMEM;
    std::string err;
    int rc;
    try {
        rc = copy_inputs(cell, atoms, basis, omega, thr, r->in, err);
    } catch (const std::bad_alloc &) {
        rc = PBC_JK_ENOMEM;
    }
    if (rc) {
        delete r;
        return rc;
    }
    // AO count from the shell list (spherical d counted as 5)
    long nbf = 0;
    for (int i = 0; i < r->in.nshell; ++i) {
        const int l = r->in.l[i];
        if (l < 0 || l > 2) {
            delete r;
            return PBC_JK_EINVAL;
        }
        nbf += (l == 2 && r->in.pure[i]) ? 5 : (l + 1) * (l + 2) / 2;
    }
    try {
        r->D.assign(D, D + nbf * nbf);
    } catch (const std::bad_alloc &) {
        delete r;
        return PBC_JK_ENOMEM;
    }
    r->J = J; r->K = K; r->E_J = E_J; r->E_K = E_K;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete r;
            return PBC_JK_EINVAL;
        }
        r->id = s->next_id++;
        r->key = s->cfg.policy == PBC_JK_SERVE_DEADLINE
                     ? std::chrono::duration<double>(r->t_submit - s->t0).count() +
                           kBuildSecPerNbf2 * (double)nbf * (double)nbf
                     : (double)r->id;
        s->reqs[r->id] = r;
        enqueue(s, r);
        s->c.submitted++;
        *ticket = r->id;
    }
    s->cv_work.notify_all();
    return 0;
}

int pbc_jk_server_wait(pbc_jk_server *s, unsigned long long ticket, pbc_jk_request_info *info)
{
    if (!s) return PBC_JK_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PBC_JK_EINVAL;
    Request *r = it->second;
    s->cv_done.wait(lk, [&] { return r->state == RState::Done; });
    s->reqs.erase(it);
    lk.unlock();
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->status = r->status;
        info->cache_hit = r->cache_hit;
        info->retries = r->retries;
        info->nbf = r->nbf;
        info->queue_ms = r->started ? ms_between(r->t_submit, r->t_start) : ms_between(r->t_submit, r->t_done);
        info->setup_ms = r->setup_ms;
        info->build_ms = r->build_ms;
        info->latency_ms = ms_between(r->t_submit, r->t_done);
        info->device_bytes = r->dev_bytes;
        std::strncpy(info->error, r->err.c_str(), sizeof info->error - 1);
    }
    const int st = r->status;
    delete r;
    return st;
}

int pbc_jk_server_cancel(pbc_jk_server *s, unsigned long long ticket)
{
    if (!s) return PBC_JK_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return PBC_JK_EINVAL;
    Request *r = it->second;
    if (r->state == RState::Building || r->state == RState::Done) return PBC_JK_EBUSY;
    r->cancel = true;
    s->cv_work.notify_all();
    return 0;
}

int pbc_jk_server_stats(pbc_jk_server *s, pbc_jk_server_counters *out)
{
    if (!s || !out) return PBC_JK_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->c;
    out->in_use = s->arena.in_use();
    out->peak_in_use = s->arena.peak();
    return 0;
}

void pbc_jk_server_destroy(pbc_jk_server *s)
{
    if (!s) return;
    std::vector<pbc_jk *> hs;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (Request *q : s->queue) {
            if (pbc_jk *h = drop_placeholder(s, q)) hs.push_back(h);
            finish(s, q, PBC_JK_ECANCELED, "server destroyed");
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (pbc_jk *h : hs) handle_delete(h);
    for (auto &kv : s->cells) {
        if (kv.second->h) handle_delete(kv.second->h);
        delete kv.second;
    }
    for (auto &kv : s->reqs) {
        if (kv.second->prepared) handle_delete(kv.second->prepared);
        delete kv.second;
    }
    delete s;
}

}  // extern "C"
