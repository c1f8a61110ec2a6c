// Continuous-batching server of Taylor-Green solves on one GPU.
//
// Admission: a request is admitted when a slot is free and a first-fit block
// of the caller's arena holds its footprint (state, Runge-Kutta register,
// face-trace / interface-flux / forcing workspace, descriptors, a device ring
// of kinetic-energy records).  Admitted solves stay resident until done.
//
// Execution: one host thread, one stream per polynomial order.  Each round it
// admits what fits, then advances every running solve by a number of
// Runge-Kutta steps sized to its order group's cost; within a step, the
// stages of all running solves of the same order run in shared launches (one
// k_grad, one batched network launch for the corrected solves, one k_resid
// per stage) on that order's stream, and the groups of different orders
// overlap on the device.  Requests that arrive while others run join them at
// the next round.  Per-solve time steps and step counts are independent;
// nothing is reduced across solves, so each result is what the solve computes
// alone.  After each round the stream is synchronised once: kinetic-energy
// records are collected, non-finite solves are failed, finished solves are
// copied out and their arena blocks released.
//
// Fallback of the learned part: a corrected solve (network forcing, Eq. (4),
// or Algorithm 1's correction) keeps a copy of its state from the start of
// each round, a state already checked healthy.  At the end of every round its
// state is checked again (finite diagnostics, kinetic energy not above
// (1 + kFallbackKeRise) times the initial value -- the Taylor-Green flow
// decays, so a rise means the forcing is driving it); when that or any of
// the round's kinetic-energy records fails, the solve returns to the copy,
// drops the records after it, and continues from there as the uncorrected
// low-order solve (Eq. (3)), flagged in its status.  A non-finite record of
// an uncorrected solve fails that solve.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "nn_internal.hpp"

namespace dgnn {

constexpr int kHist = 64;    // device KE records per solve between synchronisations
constexpr int kChunk = 16;   // steps per round of the costliest order group
constexpr int kChunkMax = 256;  // steps per round of any group
constexpr size_t kDiagDoubles = 8;
constexpr double kFallbackKeRise = 1e-3;   // relative kinetic-energy rise that ends the correction

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Foot {
    size_t q, k, ws, desc, hist, health, ckpt, total;
};

// arena layout of one solve; a corrected solve also holds the state copy of
// its fallback
static Foot foot(const Mesh& m, bool corrected) {
    Foot f;
    const size_t field = a256((size_t)5 * m.E * m.n_p * sizeof(double));
    f.q = 0;
    f.k = field;
    f.ws = 2 * field;
    f.desc = f.ws + a256(ws_layout(m).total);
    f.hist = f.desc + a256(4 * sizeof(SolveDesc));
    f.health = f.hist + a256(kHist * kDiagDoubles * sizeof(double));
    f.ckpt = f.health + a256(kDiagDoubles * sizeof(double));
    f.total = f.ckpt + (corrected ? field : 0);
    return f;
}

static dg_params request_params(const solve_request& r) {
    dg_params p;
    std::memset(&p, 0, sizeof(p));
    p.N = r.N;
    p.P = r.P;
    p.viscous = 1;
    p.L = 2.0 * M_PI;
    p.Re = r.Re;
    p.Mach = r.Mach > 0 ? r.Mach : 0.1;
    p.gamma = 1.4;
    p.Pr = 0.72;
    p.Cs = r.Cs;
    p.Pr_t = 0.6;
    p.p_ref = 1.0 / (p.gamma * p.Mach * p.Mach);
    return p;
}

struct Solve {
    uint64_t id = 0;
    solve_request req;
    Mesh mesh;
    int state = SOLVE_QUEUED;
    int error = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::atomic<int64_t> steps{0};
    int64_t n_steps = 0;
    double dt = 0;
    size_t off = 0, bytes = 0;
    double* q = nullptr;
    double* k = nullptr;
    char* ws = nullptr;
    SolveDesc* ddesc = nullptr;
    double* hist = nullptr;
    double* health = nullptr;        // diagnostics of the state at the end of a round
    double* ckpt = nullptr;          // corrected solves: state at the start of the round
    bool nn_active = false;          // the correction is applied
    bool fell_back = false;          // continued uncorrected after a failed check
    int64_t fallback_step = 0;
    int64_t ckpt_steps = 0;
    double ke0 = 0.0;
    int par = 0;
    std::vector<double> pending_t;   // times of device records not yet collected
    std::vector<double> ke;          // collected (t, KE) pairs
    std::atomic<bool> inject{false};
};

// first-fit allocator over [0, size) with coalescing
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t& off) {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
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

  private:
    std::map<size_t, size_t> free_;
};

}  // namespace dgnn

using namespace dgnn;

struct solve_server {
    char* base = nullptr;
    size_t bytes = 0;
    int max_slots = 0;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::map<uint64_t, std::unique_ptr<Solve>> solves;
    std::deque<Solve*> queue;
    std::vector<Solve*> running;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread th;
    hipStream_t st = nullptr;                 // admission work
    hipStream_t gst[dgnn::kMaxPP + 1] = {};   // one stream per order group
    Arena arena;
    double busy = 0.0;
    int64_t batches = 0;
    double* pinned = nullptr;
};

namespace dgnn {

static void fail(solve_server* S, Solve* s, int code) {
    std::lock_guard<std::mutex> lk(S->mu);
    s->state = SOLVE_FAILED;
    s->error = code;
    s->t_done = now_s();
    S->arena.release(s->off, s->bytes);
}

static int write_descs(solve_server* S, Solve* s);

// set up one admitted solve: pointers, TGV state, dt, descriptors, traces
static int admit_one(solve_server* S, Solve* s) {
    const dg_params prm = request_params(s->req);
    int rc = make_mesh(&prm, s->mesh);
    if (rc) return rc;
    const Foot f = foot(s->mesh, s->req.use_nn != 0);
    char* p = S->base + s->off;
    s->q = (double*)(p + f.q);
    s->k = (double*)(p + f.k);
    s->ws = p + f.ws;
    s->ddesc = (SolveDesc*)(p + f.desc);
    s->hist = (double*)(p + f.hist);
    s->health = (double*)(p + f.health);
    s->ckpt = s->req.use_nn ? (double*)(p + f.ckpt) : nullptr;
    s->nn_active = s->req.use_nn != 0;
    if ((rc = init_tgv_impl(s->mesh, s->q, S->st))) return rc;
    double* dout = s->hist;   // scratch for the time-step diagnostics
    if ((rc = diag_impl(s->mesh, s->q, dout, s->ws, S->st))) return rc;
    double h[kDiagDoubles];
    if (hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, S->st) != hipSuccess ||
        hipStreamSynchronize(S->st) != hipSuccess)
        return set_error(DG_EHIP, "admission readback failed");
    const double dt0 = stable_dt_from_diag(s->mesh, h, 0.4);
    if (!(dt0 > 0) || !std::isfinite(dt0)) return set_error(DG_ENONFINITE, "bad initial state");
    s->ke0 = h[0];
    s->n_steps = (int64_t)std::ceil(s->req.t_end / dt0 - 1e-12);
    if (s->n_steps < 1) s->n_steps = 1;
    s->dt = s->req.t_end / s->n_steps;
    if ((rc = write_descs(S, s))) return rc;
    if (launch_traces(s->mesh.PP, single_list(s->ddesc + 1, s->mesh.E), S->st) != hipSuccess)
        return set_error(DG_EHIP, "trace launch failed");
    // record KE(0)
    if ((rc = diag_impl(s->mesh, s->q, s->hist, s->ws, S->st))) return rc;
    if (hipStreamSynchronize(S->st) != hipSuccess) return set_error(DG_EHIP, "admission synchronise failed");
    s->pending_t.push_back(0.0);
    s->par = 0;
    s->steps = 0;
    return DG_OK;
}

// the four stage descriptors of a solve, with the correction while it is
// active: d[par] the stages, d[2 + par] the last stage of a step corrected
// after the step (Algorithm 1), whose update adds dt s(q^n)
static int write_descs(solve_server* S, Solve* s) {
    const WsLayout L = ws_layout(s->mesh);
    const bool post = s->nn_active && s->req.nn_after_step;
    const double* fbuf = s->nn_active ? (const double*)(s->ws + L.forcing) : nullptr;
    SolveDesc d[4];
    for (int p = 0; p < 4; ++p) {
        const int par = p & 1;
        std::memset(&d[p], 0, sizeof(SolveDesc));
        d[p].q = s->q;
        d[p].k = s->k;
        d[p].forcing = post ? nullptr : fbuf;
        d[p].post = (post && p >= 2) ? fbuf : nullptr;
        d[p].qtr_in = (const double*)(s->ws + (par == 0 ? L.qtr0 : L.qtr1));
        d[p].qtr_out = (double*)(s->ws + (par == 0 ? L.qtr1 : L.qtr0));
        d[p].fv = (double*)(s->ws + L.fv);
        d[p].N = s->mesh.N;
        d[p].E = s->mesh.E;
        d[p].dt = s->dt;
        d[p].ph = s->mesh.ph;
    }
    if (launch_write_descs(d, 4, s->ddesc, S->st) != hipSuccess) return set_error(DG_EHIP, "descriptor upload failed");
    return DG_OK;
}

// one Runge-Kutta step of every solve of one order group, stages batched,
// enqueued on the group's stream
static int step_group(solve_server* S, int PP, std::vector<Solve*>& v, hipStream_t st) {
    for (Solve* s : v)
        if (s->inject) {
            static const double nan_val = std::nan("");
            if (hipMemcpyAsync(s->q, &nan_val, sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
                return set_error(DG_EHIP, "inject failed");
            if (hipStreamSynchronize(st) != hipSuccess) return set_error(DG_EHIP, "inject sync failed");
            s->inject = false;
        }
    for (int stg = 0; stg < 3; ++stg) {
        for (size_t c0 = 0; c0 < v.size(); c0 += kMaxDescs) {
            const size_t cn = std::min((size_t)kMaxDescs, v.size() - c0);
            DescList dl;
            std::memset(&dl, 0, sizeof(dl));
            int blk = 0;
            for (size_t i = 0; i < cn; ++i) {
                Solve* s = v[c0 + i];
                const bool post = s->nn_active && s->req.nn_after_step;
                dl.d[i] = s->ddesc + s->par + ((post && stg == 2) ? 2 : 0);
                dl.blk[i] = blk;
                blk += s->mesh.E;
            }
            dl.blk[cn] = blk;
            dl.n = (int)cn;
            if (launch_grad(PP, dl, st) != hipSuccess) return set_error(DG_EHIP, "grad launch failed");
            // network forcing of the corrected solves, grouped by model
            std::map<const nn_model*, std::vector<NetTarget>> nets;
            for (size_t i = 0; i < cn; ++i) {
                Solve* s = v[c0 + i];
                if (!s->nn_active) continue;
                if (s->req.nn_after_step && stg != 0) continue;   // s(q^n) once, at the step start
                NetTarget t;
                t.q = s->q;
                t.out = (double*)(s->ws + ws_layout(s->mesh).forcing);
                t.E = s->mesh.E;
                t.blk_begin = 0;
                nets[s->req.model].push_back(t);
            }
            for (auto& nt : nets) {
                int rc = net_forcing_batch(nt.first, PP * PP * PP, nt.second.data(), (int)nt.second.size(), st);
                if (rc) return rc;
            }
            if (launch_resid(PP, 1, dl, kRkA[stg], kRkB[stg], stg == 0, st) != hipSuccess)
                return set_error(DG_EHIP, "resid launch failed");
        }
        for (Solve* s : v) s->par ^= 1;
    }
    for (Solve* s : v) {
        s->steps.fetch_add(1);
        if (s->steps % s->req.ke_every == 0 || s->steps == s->n_steps) {
            if ((int)s->pending_t.size() >= kHist) continue;
            int rc = diag_impl(s->mesh, s->q, s->hist + kDiagDoubles * s->pending_t.size(), s->ws, st);
            if (rc) return rc;
            s->pending_t.push_back(s->steps * s->dt);
        }
    }
    return DG_OK;
}

// cost of one step of a solve, in node-stage units (the network adds about
// as much again at every stage, less when it corrects once per step)
static double step_cost(const Solve* s) {
    return (double)s->mesh.E * s->mesh.n_p * (s->nn_active ? (s->req.nn_after_step ? 1.3 : 2.0) : 1.0);
}

// Steps of one round for each running solve.  Per order group, the group's
// costliest solve takes n_g steps, where the costliest group (by summed cost
// per step) takes kChunk and cheaper groups proportionally more, up to
// kChunkMax, so that a round takes about the same time on every stream.
// Within a group every solve gets about the same device time as that
// costliest one: a solve whose steps cost a k-th as much takes k times the
// steps (up to kChunkMax), so that a small solve batched with large ones of
// its order does not wait for as many of their steps as it needs of its own.
// Never past a solve's last step or its KE-record capacity.
static std::map<const Solve*, int64_t> round_plan(const std::map<int, std::vector<Solve*>>& groups) {
    std::map<int, double> cost;
    double cmax = 0.0;
    for (auto& g : groups) {
        double c = 0.0;
        for (Solve* s : g.second) c += step_cost(s);
        cost[g.first] = c;
        cmax = std::max(cmax, c);
    }
    std::map<const Solve*, int64_t> plan;
    for (auto& g : groups) {
        const double ng = std::max(1.0, std::min((double)kChunkMax,
                                                 std::floor(kChunk * cmax / std::max(1.0, cost[g.first]))));
        double cbig = 0.0;
        for (Solve* s : g.second) cbig = std::max(cbig, step_cost(s));
        for (Solve* s : g.second) {
            double n = std::floor(ng * cbig / std::max(1.0, step_cost(s)));
            n = std::min(n, std::max(ng, (double)kChunkMax));
            int64_t k = std::max<int64_t>((int64_t)n, 1);
            k = std::min<int64_t>(k, s->n_steps - s->steps);
            k = std::min<int64_t>(k, (int64_t)(kHist - 1 - (int)s->pending_t.size()) * s->req.ke_every);
            plan[s] = std::max<int64_t>(k, 1);
        }
    }
    return plan;
}

static bool record_finite(const double* rec) {
    bool finite = std::isfinite(rec[0]);
    for (int c = 3; c < 8; ++c) finite = finite && std::isfinite(rec[c]);
    return finite;
}

// a corrected solve's state is healthy: finite, kinetic energy not risen
static bool record_healthy(const Solve* s, const double* rec) {
    return record_finite(rec) && rec[0] <= s->ke0 * (1.0 + kFallbackKeRise);
}

// Reads the round's kinetic-energy records (and, for a corrected solve, the
// end-of-round health record).  Returns true when a corrected solve must
// fall back: its pending records are then dropped, except those at or
// before the state copy it returns to.
static bool collect(solve_server* S, Solve* s) {
    const size_t n = s->pending_t.size();
    double health[kDiagDoubles];
    const bool check = s->nn_active;
    if (n > 0 && hipMemcpy(S->pinned, s->hist, n * kDiagDoubles * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        std::lock_guard<std::mutex> lk(S->mu);
        s->error = DG_EHIP;
        return false;
    }
    if (check && hipMemcpy(health, s->health, sizeof(health), hipMemcpyDeviceToHost) != hipSuccess) {
        std::lock_guard<std::mutex> lk(S->mu);
        s->error = DG_EHIP;
        return false;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    bool bad = check && !record_healthy(s, health);
    for (size_t r = 0; r < n && check && !bad; ++r) bad = !record_healthy(s, S->pinned + r * kDiagDoubles);
    const double t_ckpt = s->ckpt_steps * s->dt;
    for (size_t r = 0; r < n; ++r) {
        const double* rec = S->pinned + r * kDiagDoubles;
        if (bad && s->pending_t[r] > t_ckpt + 0.5 * s->dt) continue;
        if (!bad && !record_finite(rec)) s->error = DG_ENONFINITE;
        s->ke.push_back(s->pending_t[r]);
        s->ke.push_back(rec[0]);
    }
    s->pending_t.clear();
    return bad;
}

// return a corrected solve to the state copy of the round start and continue
// it uncorrected from there
static int fall_back(solve_server* S, Solve* s) {
    s->nn_active = false;
    if (hipMemcpyAsync(s->q, s->ckpt, (size_t)5 * s->mesh.E * s->mesh.n_p * sizeof(double), hipMemcpyDeviceToDevice,
                       S->st) != hipSuccess)
        return set_error(DG_EHIP, "fallback restore failed");
    int rc = write_descs(S, s);
    if (rc) return rc;
    s->par = 0;
    if (launch_traces(s->mesh.PP, single_list(s->ddesc + 1, s->mesh.E), S->st) != hipSuccess)
        return set_error(DG_EHIP, "trace launch failed");
    if (hipStreamSynchronize(S->st) != hipSuccess) return set_error(DG_EHIP, "fallback synchronise failed");
    std::lock_guard<std::mutex> lk(S->mu);
    s->steps = s->ckpt_steps;
    s->fell_back = true;
    s->fallback_step = s->ckpt_steps;
    return DG_OK;
}

static void finish(solve_server* S, Solve* s) {
    if (s->req.q_out_host)
        (void)hipMemcpy(s->req.q_out_host, s->q, (size_t)5 * s->mesh.E * s->mesh.n_p * sizeof(double), hipMemcpyDeviceToHost);
    if (s->req.ke_host) {
        const size_t pairs = std::min((size_t)s->req.ke_capacity, s->ke.size() / 2);
        std::memcpy(s->req.ke_host, s->ke.data(), pairs * 2 * sizeof(double));
    }
    std::lock_guard<std::mutex> lk(S->mu);
    s->state = SOLVE_DONE;
    s->t_done = now_s();
    S->arena.release(s->off, s->bytes);
}

static void server_loop(solve_server* S) {
    (void)hipSetDevice(S->device);
    std::vector<Solve*> run;
    while (true) {
        std::vector<Solve*> admitted;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->queue.empty() || !run.empty(); });
            if (S->stop) break;
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                Solve* s = *it;
                if ((int)(run.size() + admitted.size()) >= S->max_slots) break;
                size_t off;
                if (S->arena.alloc(s->bytes, off)) {
                    s->off = off;
                    s->state = SOLVE_RUNNING;
                    s->t_admit = now_s();
                    admitted.push_back(s);
                    it = S->queue.erase(it);
                } else {
                    ++it;
                }
            }
        }
        for (Solve* s : admitted) {
            int rc = admit_one(S, s);
            if (rc) fail(S, s, rc);
            else run.push_back(s);
        }
        if (run.empty()) {
            S->cv.notify_all();
            continue;
        }
        std::map<int, std::vector<Solve*>> groups;
        for (Solve* s : run) groups[s->mesh.PP].push_back(s);
        const std::map<const Solve*, int64_t> plan = round_plan(groups);
        const double t0 = now_s();
        int rc = DG_OK;
        int64_t steps_done = 0;
        for (auto& g : groups) {
            hipStream_t gst = S->gst[g.first];
            int64_t n_g = 0;
            for (Solve* s : g.second) n_g = std::max(n_g, plan.at(s));
            // corrected solves: copy of the (already checked) state the round starts from
            for (Solve* s : g.second)
                if (s->nn_active && rc == DG_OK) {
                    s->ckpt_steps = s->steps;
                    if (hipMemcpyAsync(s->ckpt, s->q, (size_t)5 * s->mesh.E * s->mesh.n_p * sizeof(double),
                                       hipMemcpyDeviceToDevice, gst) != hipSuccess)
                        rc = set_error(DG_EHIP, "state copy failed");
                }
            // step n batches every solve that still has steps in this round
            std::vector<Solve*> active;
            for (int64_t n = 0; n < n_g && rc == DG_OK; ++n) {
                active.clear();
                for (Solve* s : g.second)
                    if (plan.at(s) > n) active.push_back(s);
                rc = step_group(S, g.first, active, gst);
            }
            for (Solve* s : g.second)
                if (s->nn_active && rc == DG_OK) rc = diag_impl(s->mesh, s->q, s->health, s->ws, gst);
            steps_done = std::max(steps_done, n_g);
        }
        for (auto& g : groups) (void)hipStreamSynchronize(S->gst[g.first]);
        const double t1 = now_s();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->busy += t1 - t0;
            S->batches += steps_done;
        }
        std::vector<Solve*> keep;
        for (Solve* s : run) {
            const bool back = collect(S, s);
            if (back && rc == DG_OK) {
                const int frc = fall_back(S, s);
                if (frc) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    s->error = frc;
                }
            }
            int err;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (rc != DG_OK) s->error = rc;
                err = s->error;
            }
            if (err) fail(S, s, err);
            else if (s->steps >= s->n_steps) finish(S, s);
            else keep.push_back(s);
        }
        run.swap(keep);
        S->cv.notify_all();
    }
    S->cv.notify_all();
}

}  // namespace dgnn

extern "C" {

size_t solve_footprint(int32_t P, int32_t N, int32_t use_nn) {
    if (P < DG_MIN_ORDER || P > DG_MAX_ORDER || N < 1 || N > 1024) return 0;
    Mesh m;
    std::memset(&m, 0, sizeof(m));
    m.N = N;
    m.P = P;
    m.PP = P + 1;
    m.E = N * N * N;
    m.n_p = m.PP * m.PP * m.PP;
    m.n_f = m.PP * m.PP;
    return foot(m, use_nn != 0).total;
}

int solve_server_create(void* arena, size_t arena_bytes, int32_t max_slots, solve_server** out) {
    if (!out) return set_error(DG_EINVAL, "null output handle");
    *out = nullptr;
    if (!arena || (((uintptr_t)arena) & 255)) return set_error(DG_EINVAL, "arena must be non-null and 256-byte aligned");
    if (max_slots < 1 || max_slots > 4096) return set_error(DG_EINVAL, "max_slots outside [1, 4096]");
    solve_server* S = new solve_server;
    S->base = (char*)arena;
    S->bytes = arena_bytes & ~(size_t)255;
    S->max_slots = max_slots;
    S->arena.reset(S->bytes);
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return set_error(DG_EHIP, "hipGetDevice failed");
    }
    if (hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) != hipSuccess) {
        delete S;
        return set_error(DG_EHIP, "stream creation failed");
    }
    for (int pp = DG_MIN_ORDER + 1; pp <= kMaxPP; ++pp)
        if (hipStreamCreateWithFlags(&S->gst[pp], hipStreamNonBlocking) != hipSuccess) {
            for (int q = DG_MIN_ORDER + 1; q < pp; ++q) (void)hipStreamDestroy(S->gst[q]);
            (void)hipStreamDestroy(S->st);
            delete S;
            return set_error(DG_EHIP, "stream creation failed");
        }
    if (hipHostMalloc((void**)&S->pinned, kHist * kDiagDoubles * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipStreamDestroy(S->st);
        for (int pp = DG_MIN_ORDER + 1; pp <= kMaxPP; ++pp) (void)hipStreamDestroy(S->gst[pp]);
        delete S;
        return set_error(DG_EHIP, "pinned buffer allocation failed");
    }
    S->th = std::thread(server_loop, S);
    *out = S;
    return DG_OK;
}

int solve_submit(solve_server* S, const solve_request* r, uint64_t* id) {
    if (!S || !r || !id) return set_error(DG_EINVAL, "null argument");
    if (!(r->Re > 0) || !(r->t_end > 0) || !std::isfinite(r->t_end) || r->ke_every < 1 || r->Cs < 0)
        return set_error(DG_EINVAL, "invalid request parameters");
    if (r->ke_host && r->ke_capacity < 0) return set_error(DG_EINVAL, "negative KE capacity");
    if (r->nn_after_step != 0 && r->nn_after_step != 1) return set_error(DG_EINVAL, "nn_after_step must be 0 or 1");
    Mesh m;
    dg_params p = request_params(*r);
    int rc = make_mesh(&p, m);
    if (rc) return rc;
    if (r->use_nn) {
        if (!r->model) return set_error(DG_EINVAL, "use_nn without a model");
        if ((rc = net_check_mesh(r->model, m))) return rc;
    }
    const size_t need = foot(m, r->use_nn != 0).total;
    if (need > S->bytes) return set_error(DG_ENOSPC, "request needs %zu bytes, arena holds %zu", need, S->bytes);
    auto s = std::make_unique<Solve>();
    s->req = *r;
    s->mesh = m;
    s->bytes = need;
    s->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return set_error(DG_EINVAL, "server is shutting down");
        s->id = S->next_id++;
        *id = s->id;
        S->queue.push_back(s.get());
        S->solves[s->id] = std::move(s);
    }
    S->cv.notify_all();
    return DG_OK;
}

int solve_poll(solve_server* S, uint64_t id, solve_status* st) {
    if (!S || !st) return set_error(DG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->solves.find(id);
    if (it == S->solves.end()) return set_error(DG_ENOENT, "unknown request %llu", (unsigned long long)id);
    const Solve* s = it->second.get();
    std::memset(st, 0, sizeof(*st));
    st->state = s->state;
    st->error = s->error;
    st->steps = s->steps;
    st->n_steps = s->n_steps;
    st->ke_count = (int32_t)std::min((size_t)std::max(0, s->req.ke_capacity), s->ke.size() / 2);
    st->fallback = s->fell_back ? 1 : 0;
    st->fallback_step = s->fell_back ? s->fallback_step : -1;
    st->t = s->steps * s->dt;
    st->dt = s->dt;
    st->queue_s = s->state == SOLVE_QUEUED ? 0.0 : s->t_admit - s->t_submit;
    st->latency_s = (s->state == SOLVE_DONE || s->state == SOLVE_FAILED) ? s->t_done - s->t_submit : 0.0;
    st->dof_updates = (int64_t)3 * s->steps * s->mesh.E * s->mesh.n_p;
    return (s->state == SOLVE_DONE || s->state == SOLVE_FAILED) ? DG_OK : DG_EAGAIN;
}

int solve_server_drain(solve_server* S) {
    if (!S) return set_error(DG_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv.wait(lk, [&] {
        if (!S->queue.empty()) return false;
        for (auto& kv : S->solves)
            if (kv.second->state == SOLVE_RUNNING) return false;
        return true;
    });
    return DG_OK;
}

int solve_inject_nan(solve_server* S, uint64_t id) {
    if (!S) return set_error(DG_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->solves.find(id);
    if (it == S->solves.end()) return set_error(DG_ENOENT, "unknown request");
    it->second->inject = true;
    return DG_OK;
}

int solve_server_stats(solve_server* S, double* busy_s, int64_t* batches) {
    if (!S) return set_error(DG_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (busy_s) *busy_s = S->busy;
    if (batches) *batches = S->batches;
    return DG_OK;
}

void solve_server_free(solve_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    (void)hipStreamSynchronize(S->st);
    (void)hipStreamDestroy(S->st);
    for (int pp = DG_MIN_ORDER + 1; pp <= kMaxPP; ++pp) {
        (void)hipStreamSynchronize(S->gst[pp]);
        (void)hipStreamDestroy(S->gst[pp]);
    }
    (void)hipHostFree(S->pinned);
    delete S;
}

}  // extern "C"
