// Continuous-batching request loop over resident encoding matrices.
//
// Each registered matrix (a tvcs_handle) is a group with a fixed number of image
// slots: its batch workspace and captured iteration graph are those of a batched
// solve over all slots, on the handle's own stream.  Groups run independently:
// a scheduling round (tvcs_server_step)
//   1. takes every group whose previous replay has finished: retires the slots
//      whose image met its stop rule (eq. (stop)) or its cap, admits queued
//      requests into free slots (copies f, sets the slot's state, u^0 = A^T f for
//      the new slots only, q^{-1} = D u^0 for IADM), allocating a group's slots on
//      first use only if the device memory counted against the budget allows it,
//      and relaunches the group's graph (10 iterations) if it holds requests;
//   2. returns once at least one running group has finished its replay (no group
//      waits for another's).
// Slots that finish mid-replay are predicated off on the device, so a request's
// iterations and result do not depend on when it was admitted or on its
// neighbours: every reduction order is fixed by (n, m) alone.
//
// Budget: a group that does not fit waits; after kStarveRounds rounds of waiting,
// the other groups stop admitting new requests, finish the ones they hold, and
// give their memory back, so the wait of every matrix is bounded by about one
// request's iteration cap.
#include <deque>
#include <unordered_map>
#include <vector>

#include <chrono>
#include <thread>

#include "solver.h"

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

constexpr int kStarveRounds = 4;   // rounds a group may wait for memory before others drain

struct SrvRequest {
    int matrix = 0;
    std::vector<float> f;
    double tol = 0.0;
    int maxit = 1;
    bool done = false;
    double t_admit = 0.0;
    std::vector<float> u;
    tvcs_stats st{};
};

struct SrvGroup {
    tvcs_ctx *h = nullptr;
    bool ready = false;                 // slots allocated and graph built
    bool inflight = false;              // a replay and its state copy are queued
    hipEvent_t done = nullptr;          // recorded after the state copy of the replay
    std::vector<long long> slot;        // request id per slot, -1 if free
    std::deque<long long> queue;
    bool busy() const {
        for (long long r : slot)
            if (r >= 0) return true;
        return false;
    }
};

}  // namespace

struct tvcs_server {
    size_t budget = 0;
    int slots = 0;
    double mu = 0, beta = 0;
    unsigned flags = 0;
    std::vector<SrvGroup> groups;
    std::unordered_map<long long, SrvRequest> reqs;
    long long next_id = 0;
    int starving = -1;       // group waiting for memory (first in line), or -1
    int starve_rounds = 0;
    double a_bytes = 0.0;    // bytes of A the launched replays stream (two products per iteration)

    ~tvcs_server() {
        for (SrvGroup &g : groups) {
            if (g.h) (void)hipStreamSynchronize(g.h->work);
            if (g.done) (void)hipEventDestroy(g.done);
        }
    }

    size_t counted_bytes() const {
        size_t b = 0;
        for (const SrvGroup &g : groups) b += g.h->device_bytes();
        return b;
    }

    bool draining() const { return starving >= 0 && starve_rounds > kStarveRounds; }

    // allocate group gi's slots if the budget allows (releasing idle groups first)
    bool make_ready(int gi) {
        SrvGroup &g = groups[gi];
        if (g.ready) return true;
        tvcs_ctx *h = g.h;
        const size_t need = h->storage_bytes() + h->workspace_bytes(slots) + h->admission_bytes(slots);
        auto other = [&] { return counted_bytes() - h->device_bytes(); };
        if (budget && other() + need > budget) {
            for (size_t j = 0; j < groups.size(); ++j) {
                SrvGroup &o = groups[j];
                if ((int)j == gi || !o.ready || o.inflight || o.busy()) continue;
                if (!o.queue.empty() && !draining()) continue;
                o.h->release_workspace();
                o.ready = false;
                if (other() + need <= budget) break;
            }
            if (other() + need > budget) return false;
        }
        h->begin_call();
        h->ensure_workspace(slots);
        h->adm_F.ensure(sizeof(float) * (size_t)h->capP * h->m);
        h->adm_U.ensure(sizeof(float) * (size_t)h->capP * h->N);
        const double tau = h->tau();
        const double c = mu / (beta * tau);
        h->ensure_denominators(c);
        // every slot starts free and inactive
        for (int s = 0; s < slots; ++s)
            h->host_state[s] = ImgState{0, 0, TVCS_OK, 1, 0.0, 0.0, 0.0, 0.0, {1, 1}, 0, 0};
        TVCS_HIP(hipMemcpyAsync(h->state.p, h->host_state, sizeof(ImgState) * slots,
                                hipMemcpyHostToDevice, h->work));
        h->build_graph(slots, flags & TVCS_IADM, beta, c, mu / beta);
        TVCS_HIP(hipStreamSynchronize(h->work));
        if (!g.done) TVCS_HIP(hipEventCreateWithFlags(&g.done, hipEventDisableTiming));
        g.slot.assign(slots, -1);
        g.ready = true;
        return true;
    }

    // results of the slots of an idle group whose image has stopped
    void retire(int gi) {
        SrvGroup &g = groups[gi];
        tvcs_ctx *h = g.h;
        const double t = now_ms();
        for (int s = 0; s < slots; ++s) {
            if (g.slot[s] < 0) continue;
            const ImgState &is = h->host_state[s];
            if (is.active) continue;
            SrvRequest &r = reqs[g.slot[s]];
            r.u.resize((size_t)h->N);
            TVCS_HIP(hipMemcpyAsync(r.u.data(), h->U.as<float>() + (size_t)s * h->N,
                                    sizeof(float) * h->N, hipMemcpyDeviceToHost, h->work));
            r.st.iters = is.iters;
            r.st.status = is.status;
            r.st.rel_change = is.rel;
            r.st.fresh_iters = h->lowprec() ? is.fresh : 0;
            h->tiles_out(r.st.tiles);
            r.st.objective = 0.0;
            r.st.tau = h->tau();
            r.st.ms = (float)(t - r.t_admit);
            r.done = true;
            r.f.clear();
            r.f.shrink_to_fit();
            g.slot[s] = -1;
        }
        TVCS_HIP(hipStreamSynchronize(h->work));
    }

    // queued requests of an idle, ready group into its free slots
    void admit(int gi) {
        SrvGroup &g = groups[gi];
        if (g.queue.empty() || (draining() && gi != starving)) return;
        tvcs_ctx *h = g.h;
        std::vector<int> fresh;
        for (int s = 0; s < slots && !g.queue.empty(); ++s) {
            if (g.slot[s] >= 0) continue;
            const long long id = g.queue.front();
            g.queue.pop_front();
            g.slot[s] = id;
            fresh.push_back(s);
        }
        if (fresh.empty()) return;
        const int N = h->N, m = h->m, nf = (int)fresh.size();
        float *U = h->U.as<float>();
        ImgState *st = h->state.as<ImgState>();
        // u^0 = A^T f for the new slots only: their f staged contiguously in adm_F
        // (capP rows, the padded batch the products read), the product into adm_U
        float *stage = h->adm_F.as<float>(), *T = h->adm_U.as<float>();
        const double t = now_ms();
        for (int j = 0; j < nf; ++j) {
            const int s = fresh[j];
            SrvRequest &r = reqs[g.slot[s]];
            r.t_admit = t;
            h->load_measurements(r.f.data(), s, 1);
            TVCS_HIP(hipMemcpyAsync(stage + (size_t)j * m, r.f.data(), sizeof(float) * m,
                                    hipMemcpyHostToDevice, h->work));
            h->host_state[s] = ImgState{0, 1, TVCS_OK, r.maxit, 0.0, 0.0, 0.0, r.tol, {1, 1}, 0, 0};
            TVCS_HIP(hipMemcpyAsync(st + s, h->host_state + s, sizeof(ImgState),
                                    hipMemcpyHostToDevice, h->work));
        }
        if (h->dct()) {
            // the partial DCT keeps f in its pass order: A^T f from the slots' rows of F
            h->apply_At_full(h->capP, slots, h->F.as<float>(), T, nullptr);
            for (int s : fresh)
                TVCS_HIP(hipMemcpyAsync(U + (size_t)s * N, T + (size_t)s * N, sizeof(float) * N,
                                        hipMemcpyDeviceToDevice, h->work));
        } else {
            h->apply_At_full(h->padded(nf), nf, stage, T, nullptr);
            for (int j = 0; j < nf; ++j)
                TVCS_HIP(hipMemcpyAsync(U + (size_t)fresh[j] * N, T + (size_t)j * N,
                                        sizeof(float) * N, hipMemcpyDeviceToDevice, h->work));
        }
        for (int s : fresh)
            if (flags & TVCS_IADM)   // replays start on an even iteration: q is read from Q0
                launch_init_q(h->n, 1, U + (size_t)s * N, nullptr, beta,
                              h->Q0.as<float2>() + (size_t)s * N, h->work);
        h->seed_dct_rows(slots);   // partial DCT: row transforms of every slot's u
    }

    void launch(int gi) {
        SrvGroup &g = groups[gi];
        TVCS_HIP(hipGraphLaunch(g.h->exec, g.h->work));
        a_bytes += 2.0 * kGraphIters * (double)g.h->a_copy_bytes();
        TVCS_HIP(hipMemcpyAsync(g.h->host_state, g.h->state.p, sizeof(ImgState) * slots,
                                hipMemcpyDeviceToHost, g.h->work));
        TVCS_HIP(hipEventRecord(g.done, g.h->work));
        g.inflight = true;
    }

    // a running group whose replay has ended (its host state is then current)
    bool finished(int gi) {
        SrvGroup &g = groups[gi];
        if (!g.inflight) return false;
        const hipError_t e = hipEventQuery(g.done);
        if (e == hipErrorNotReady) return false;
        TVCS_HIP(e);
        g.inflight = false;
        return true;
    }

    // every idle group: retire, admit, relaunch
    void schedule_idle() {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            SrvGroup &g = groups[gi];
            if (g.inflight && !finished((int)gi)) continue;
            if (g.ready && g.busy()) retire((int)gi);
            if (!g.queue.empty() && !g.ready) {
                if (make_ready((int)gi)) {
                    if (starving == (int)gi) starving = -1;
                } else if (starving < 0) {
                    starving = (int)gi;
                    starve_rounds = 0;
                }
            }
            if (g.ready) admit((int)gi);
            if (g.ready && g.busy()) launch((int)gi);
        }
    }

    bool any_inflight() const {
        for (const SrvGroup &g : groups)
            if (g.inflight) return true;
        return false;
    }

    int step() {
        schedule_idle();
        // a group checked for room before another's replay was seen to end may fit
        // now that every group is idle: one more pass before giving up
        if (!any_inflight() && pending() > 0) schedule_idle();
        if (starving >= 0) ++starve_rounds;
        if (!any_inflight()) {
            if (pending() > 0)
                fail(TVCS_ENOMEM, "queued requests cannot be admitted: one matrix's slots do not "
                                  "fit in the device-memory budget");
            return 0;
        }
        // return once some running group has finished its replay
        for (;;) {
            for (size_t gi = 0; gi < groups.size(); ++gi)
                if (groups[gi].inflight && hipEventQuery(groups[gi].done) != hipErrorNotReady)
                    return pending();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    }

    int pending() const {
        int p = 0;
        for (const SrvGroup &g : groups) {
            p += (int)g.queue.size();
            for (long long r : g.slot) p += r >= 0;
        }
        return p;
    }

    // wait for every running replay (and retire what it finished)
    void drain_all() {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            SrvGroup &g = groups[gi];
            if (!g.inflight) continue;
            TVCS_HIP(hipEventSynchronize(g.done));
            g.inflight = false;
            retire((int)gi);
        }
    }
};

extern "C" {

tvcs_server *tvcs_server_create(size_t hbm_budget, int slots, double mu, double beta,
                                unsigned flags) {
    tvcs_server *out = nullptr;
    const int rc = guarded([&] {
        if (slots < 1 || slots > 1024) fail(TVCS_EINVAL, "slots must be in [1, 1024]");
        if (!(mu > 0) || !(beta > 0) || !std::isfinite(mu) || !std::isfinite(beta))
            fail(TVCS_EINVAL, "mu and beta must be positive and finite");
        if (flags & ~TVCS_IADM) fail(TVCS_EINVAL, "only TVCS_IADM is a server flag");
        out = new tvcs_server();
        out->budget = hbm_budget;
        out->slots = slots;
        out->mu = mu;
        out->beta = beta;
        out->flags = flags;
        return TVCS_OK;
    });
    return rc == TVCS_OK ? out : nullptr;
}

int tvcs_server_add_matrix(tvcs_server *s, tvcs_handle h) {
    return guarded([&] {
        if (!s || !h) fail(TVCS_EINVAL, "null server or handle");
        for (const SrvGroup &g : s->groups)
            if (g.h == h) fail(TVCS_EINVAL, "matrix already registered");
        SrvGroup g;
        g.h = h;
        (void)hipStreamSynchronize(h->work);
        h->release_workspace();   // the slots are allocated on first admission
        s->groups.push_back(std::move(g));
        return (int)s->groups.size() - 1;
    });
}

long long tvcs_server_submit(tvcs_server *s, int matrix, const float *f, double tol, int maxit) {
    long long id = -1;
    const int rc = guarded([&] {
        if (!s || !f) fail(TVCS_EINVAL, "null server or f");
        if (matrix < 0 || matrix >= (int)s->groups.size()) fail(TVCS_EINVAL, "unknown matrix id");
        if (!(tol >= 0) || !std::isfinite(tol)) fail(TVCS_EINVAL, "tol must be >= 0");
        if (maxit < 1) fail(TVCS_EINVAL, "maxit must be >= 1");
        SrvGroup &g = s->groups[matrix];
        SrvRequest r;
        r.matrix = matrix;
        r.tol = tol;
        r.maxit = maxit;
        r.f.resize((size_t)g.h->m);
        TVCS_HIP(hipMemcpy(r.f.data(), f, sizeof(float) * g.h->m, hipMemcpyDefault));
        id = s->next_id++;
        s->reqs.emplace(id, std::move(r));
        g.queue.push_back(id);
        return TVCS_OK;
    });
    return rc == TVCS_OK ? id : (long long)rc;
}

int tvcs_server_step(tvcs_server *s) {
    return guarded([&] {
        if (!s) fail(TVCS_EINVAL, "null server");
        return s->step();
    });
}

int tvcs_server_result(tvcs_server *s, long long request, float *u, tvcs_stats *st) {
    return guarded([&] {
        if (!s) fail(TVCS_EINVAL, "null server");
        auto it = s->reqs.find(request);
        if (it == s->reqs.end()) fail(TVCS_EINVAL, "unknown request id");
        if (!it->second.done) return 0;
        if (u)
            TVCS_HIP(hipMemcpy(u, it->second.u.data(), sizeof(float) * it->second.u.size(),
                               hipMemcpyDefault));
        if (st) *st = it->second.st;
        s->reqs.erase(it);
        return 1;
    });
}

int tvcs_server_pending(tvcs_server *s) { return s ? s->pending() : TVCS_EINVAL; }

size_t tvcs_server_device_bytes(tvcs_server *s) { return s ? s->counted_bytes() : 0; }

double tvcs_server_a_bytes(tvcs_server *s) { return s ? s->a_bytes : -1.0; }

void tvcs_server_destroy(tvcs_server *s) {
    if (!s) return;
    delete s;   // the destructor waits for every group's stream
}

}  // extern "C"
