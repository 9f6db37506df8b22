// Continuous-batching solve server on one device.
//
// Requests (voxel grid, densities, fixity, 1..4 load vectors, solve options)
// are queued on submit.  A scheduler thread admits the oldest queued request
// as soon as a slot is idle and the HBM ledger can hold the request's
// footprint; each slot owns a stream (default priority) and a device-resident
// mesh that is kept across requests and reused when the next request has the
// same grid, so consecutive same-size requests only upload densities, fixity
// and loads.  Slots run concurrently, so the kernels of different requests
// overlap on the device; a request that fails (bad input, non-convergence)
// completes with its own status and does not affect the others.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "afd_internal.h"

namespace {

double clock_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t ticket;
    afd_mesh_desc desc;
    std::vector<double> rho, F, x0;
    std::vector<uint8_t> fixed;
    std::vector<int32_t> pairs;
    int nrhs;
    afd_solve_opts opts;
    afd_result* res;
    uint64_t bytes;
    double t_submit;
};

struct Slot {
    afd_context* ctx = nullptr;
    afd_mesh* mesh = nullptr;
    afd_mesh_desc desc{};
    uint64_t mesh_bytes = 0;     // ledger charge of the resident mesh
    std::unique_ptr<Req> job;
    std::thread th;
    bool busy = false;
};

bool same_desc(const afd_mesh_desc& a, const afd_mesh_desc& b) { return memcmp(&a, &b, sizeof(a)) == 0; }

}  // namespace

struct afd_server {
    int device = 0;
    uint64_t budget = 0;
    uint64_t used = 0;  // bytes charged: resident meshes of all slots
    double t0 = 0;
    std::vector<Slot> slots;
    std::deque<std::unique_ptr<Req>> queue;
    std::map<uint64_t, int> status;  // ticket -> AFD_PENDING / final status
    uint64_t next_ticket = 1;
    bool stop = false;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_slot;
    std::thread sched;
};

namespace {

uint64_t footprint_of(const afd_mesh_desc& d, int nrhs, int precision) {
    // estimate without a device mesh: same formula as afd_mesh_footprint
    const uint64_t nn = (uint64_t)(d.nx + 1) * (d.ny + 1) * (d.nz + 1), ne = (uint64_t)d.nx * d.ny * d.nz,
                   nd = 3 * nn;
    uint64_t b = ne * 12 + nn * 13 + nd + 576 * 8 + (uint64_t)4 * nd * 8 * 8;
    afd::Grid g{};
    g.nx = d.nx, g.ny = d.ny, g.nz = d.nz;
    int64_t ntr = 0;
    const int64_t ntm = afd::tile_layout_sizes(g, &ntr);
    b += (uint64_t)ntr * 12 + (uint64_t)ntm * 2;
    if (precision == AFD_MIXED) b += (uint64_t)4 * nd * 4 * 8;
    if (ne <= (uint64_t)afd::PERSISTENT_MAX_ELEMS) b += (uint64_t)4 * ne * 24 * 8;  // persistent form's element buffer
    if (d.bx > 0 && d.by > 0 && d.bz > 0) {
        int nb[3] = {(d.nx + d.bx - 1) / d.bx, (d.ny + d.by - 1) / d.by, (d.nz + d.bz - 1) / d.bz};
        std::sort(nb, nb + 3);
        const int w = 6 * (nb[0] * nb[1] + nb[0] + 1) + 5;
        const int nc = 6 * nb[0] * nb[1] * nb[2];
        const int P = afd::choose_coarse_P(nc, w);
        const int K = (nc + P - 1) / P;
        b += (uint64_t)P * P * K * 8 * 6 + (uint64_t)P * P * 8 * 2 + (uint64_t)K * P * 8 * 14;
        b += (uint64_t)P * P * K * 4 * 4;                             // FP32 copies of the solve matrices
    }
    (void)nrhs;
    return b + (64ull << 20);  // partials, radix scratch, allocator slack
}

void run_job(afd_server* S, int si) {
    Slot& sl = S->slots[si];
    Req& r = *sl.job;
    afd_result* res = r.res;
    res->t_start = clock_s() - S->t0;
    int rc = AFD_OK;
    if (sl.mesh && !same_desc(sl.desc, r.desc)) {
        afd_mesh_destroy(sl.mesh);
        sl.mesh = nullptr;
    }
    if (!sl.mesh) rc = afd_mesh_create(sl.ctx, &r.desc, &sl.mesh);
    if (rc == AFD_OK) {
        sl.desc = r.desc;
        rc = afd_mesh_set_scale(sl.mesh, r.rho.data(), (int64_t)r.rho.size(), AFD_MEM_HOST);
    }
    if (rc == AFD_OK) rc = afd_mesh_set_fixed(sl.mesh, r.fixed.data(), (int64_t)r.fixed.size(), AFD_MEM_HOST);
    std::vector<double> U;
    std::vector<afd_solve_stats> st(r.nrhs);
    if (rc == AFD_OK) {
        afd_solve_opts o = r.opts;
        o.mem_kind = AFD_MEM_HOST;
        o.pairs = r.pairs.empty() ? nullptr : r.pairs.data();
        o.x0 = r.x0.empty() ? nullptr : r.x0.data();
        double* Uout = res->U;
        if (!Uout) {
            U.resize(r.F.size());
            Uout = U.data();
        }
        rc = afd_solve(sl.mesh, &o, r.nrhs, r.F.data(), Uout, (double*)res->J, nullptr, st.data());
        if (res->stats) memcpy(res->stats, st.data(), st.size() * sizeof(afd_solve_stats));
    }
    if (rc == AFD_E_OOM || rc == AFD_E_HIP) {  // do not keep a mesh in an unknown state
        if (sl.mesh) afd_mesh_destroy(sl.mesh);
        sl.mesh = nullptr;
    }
    res->t_done = clock_s() - S->t0;
    res->status = rc;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        // a slot without a mesh (never created, or freed above) holds no memory
        if (!sl.mesh) {
            S->used -= sl.mesh_bytes;
            sl.mesh_bytes = 0;
        }
        S->status[r.ticket] = rc;
        sl.job.reset();
        sl.busy = false;
    }
    S->cv_done.notify_all();
    S->cv_sched.notify_all();
}

void slot_loop(afd_server* S, int si) {
    (void)hipSetDevice(S->device);
    Slot& sl = S->slots[si];
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_slot.wait(lk, [&] { return S->stop || (sl.busy && sl.job); });
            if (!sl.job) return;  // stop requested and nothing assigned
        }
        run_job(S, si);
    }
}

void sched_loop(afd_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_sched.wait(lk, [&] {
            if (S->queue.empty()) return S->stop;
            for (auto& s : S->slots)
                if (!s.busy) return true;
            return false;
        });
        if (S->queue.empty() && S->stop) return;
        // admit the oldest request into an idle slot whose resident mesh can be
        // replaced within the budget; prefer a slot that already holds its grid
        Req& head = *S->queue.front();
        int pick = -1;
        for (size_t i = 0; i < S->slots.size(); ++i)
            if (!S->slots[i].busy && S->slots[i].mesh && same_desc(S->slots[i].desc, head.desc)) pick = (int)i;
        if (pick < 0) {
            // idle slots ordered: empty first, then the one holding the most memory
            uint64_t best_free = 0;
            for (size_t i = 0; i < S->slots.size(); ++i) {
                Slot& s = S->slots[i];
                if (s.busy) continue;
                const uint64_t after = S->used - s.mesh_bytes + head.bytes;
                if (after <= S->budget && (pick < 0 || s.mesh_bytes > best_free)) {
                    pick = (int)i;
                    best_free = s.mesh_bytes;
                }
            }
            if (pick < 0) {
                // evict the idle resident meshes to make room: their charges are
                // released under the lock, the meshes are freed (hipFree) outside
                // it, by this thread, before any slot is given new work; then retry
                std::vector<afd_mesh*> evict;
                bool released = false;
                for (auto& s : S->slots)
                    if (!s.busy && s.mesh_bytes > 0) {
                        if (s.mesh) evict.push_back(s.mesh);
                        s.mesh = nullptr;
                        S->used -= s.mesh_bytes;
                        s.mesh_bytes = 0;
                        released = true;
                    }
                if (released) {
                    lk.unlock();
                    for (afd_mesh* mh : evict) afd_mesh_destroy(mh);
                    lk.lock();
                    continue;
                }
                S->cv_sched.wait(lk);  // nothing idle to evict: wait for a running request to finish
                continue;
            }
        }
        Slot& s = S->slots[pick];
        S->used = S->used - s.mesh_bytes + head.bytes;
        s.mesh_bytes = head.bytes;
        s.job = std::move(S->queue.front());
        S->queue.pop_front();
        s.busy = true;
        S->cv_slot.notify_all();
    }
}

}  // namespace

extern "C" {

int afd_server_create(afd_context* ctx, uint64_t budget, int32_t max_slots, afd_server** out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 16) {
        afd::set_error("server_create: bad argument (1..16 slots)");
        return AFD_E_INVALID_ARG;
    }
    *out = nullptr;
    int dev = 0;
    AFD_HIP_TRY(hipGetDevice(&dev));
    afd_server* S = new afd_server();
    S->device = dev;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete S;
            afd::set_error("hipMemGetInfo failed");
            return AFD_E_HIP;
        }
        budget = (uint64_t)(0.9 * (double)fr);
    }
    S->budget = budget;
    S->t0 = clock_s();
    S->slots.resize(max_slots);
    for (auto& s : S->slots) {
        int rc = afd_context_create(dev, nullptr, &s.ctx);
        if (rc != AFD_OK) {
            for (auto& q : S->slots)
                if (q.ctx) afd_context_destroy(q.ctx);
            delete S;
            return rc;
        }
        // slots record and replay their iteration graphs like any context:
        // the library's device allocations and frees (a slot creating or
        // dropping a mesh) and graph recordings exclude one another through
        // one process-wide lock, so no capture sees a device-synchronising
        // free from another slot
    }
    for (int i = 0; i < max_slots; ++i) S->slots[i].th = std::thread(slot_loop, S, i);
    S->sched = std::thread(sched_loop, S);
    *out = S;
    return AFD_OK;
}

int afd_server_submit(afd_server* S, const afd_request* q, afd_result* res, uint64_t* ticket) {
    if (!S || !q || !res || !ticket || !q->rho || !q->fixed || !q->F || q->nrhs < 1 || q->nrhs > 4 ||
        q->opts.npairs < 0 || q->nrhs + q->opts.npairs > 16 || (q->opts.npairs > 0 && !q->opts.pairs) ||
        !(q->opts.rtol > 0) || q->opts.max_iter < 1 ||
        (q->opts.precision != AFD_FP64 && q->opts.precision != AFD_MIXED)) {
        afd::set_error("server_submit: bad request");
        return AFD_E_INVALID_ARG;
    }
    for (int p = 0; p < 2 * q->opts.npairs; ++p)
        if (q->opts.pairs[p] < 0 || q->opts.pairs[p] >= q->nrhs) {
            afd::set_error("server_submit: pair index out of range");
            return AFD_E_INVALID_ARG;
        }
    AFD_TRY(afd::validate_desc(q->desc));
    const afd_mesh_desc& d = q->desc;
    const int64_t ne = (int64_t)d.nx * d.ny * d.nz, nd = 3 * (int64_t)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    auto r = std::make_unique<Req>();
    r->desc = d;
    r->rho.assign(q->rho, q->rho + ne);
    r->fixed.assign(q->fixed, q->fixed + nd);
    r->F.assign(q->F, q->F + nd * q->nrhs);
    if (q->opts.npairs > 0) r->pairs.assign(q->opts.pairs, q->opts.pairs + 2 * q->opts.npairs);
    if (q->opts.x0) r->x0.assign(q->opts.x0, q->opts.x0 + nd * q->nrhs);
    r->nrhs = q->nrhs;
    r->opts = q->opts;
    r->res = res;
    r->bytes = footprint_of(d, q->nrhs, q->opts.precision);
    res->status = AFD_PENDING;
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->bytes > S->budget) {
        afd::set_error("server_submit: request footprint exceeds the HBM budget");
        return AFD_E_OVER_BUDGET;
    }
    r->t_submit = clock_s() - S->t0;
    res->t_submit = r->t_submit;
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->status[r->ticket] = AFD_PENDING;
    S->queue.push_back(std::move(r));
    S->cv_sched.notify_all();
    return AFD_OK;
}

int afd_server_poll(afd_server* S, uint64_t ticket) {
    if (!S) return AFD_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->status.find(ticket);
    if (it == S->status.end()) {
        afd::set_error("server_poll: unknown ticket");
        return AFD_E_INVALID_ARG;
    }
    return it->second;
}

int afd_server_wait(afd_server* S, uint64_t ticket, double timeout_s) {
    if (!S) return AFD_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto done = [&] {
        auto it = S->status.find(ticket);
        return it == S->status.end() || it->second != AFD_PENDING;
    };
    if (timeout_s < 0) S->cv_done.wait(lk, done);
    else S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    auto it = S->status.find(ticket);
    if (it == S->status.end()) {
        afd::set_error("server_wait: unknown ticket");
        return AFD_E_INVALID_ARG;
    }
    return it->second;
}

double afd_server_clock(afd_server* S) { return S ? clock_s() - S->t0 : 0.0; }

void afd_server_destroy(afd_server* S) {
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        // let queued and running work finish
        S->cv_done.wait(lk, [&] {
            if (!S->queue.empty()) return false;
            for (auto& s : S->slots)
                if (s.busy) return false;
            return true;
        });
        S->stop = true;
    }
    S->cv_sched.notify_all();
    S->cv_slot.notify_all();
    if (S->sched.joinable()) S->sched.join();
    for (auto& s : S->slots)
        if (s.th.joinable()) s.th.join();
    for (auto& s : S->slots) {
        if (s.mesh) afd_mesh_destroy(s.mesh);
        if (s.ctx) afd_context_destroy(s.ctx);
    }
    delete S;
}

}  // extern "C"
