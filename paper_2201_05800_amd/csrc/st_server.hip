// st_server.hip -- continuous batching of independent slab solves.
//
// A scheduler thread owns one HIP stream.  Every tick it
//   1. admits queued requests while a slot is free and their device
//      footprint fits the HBM budget (first-fit sub-allocation of one arena),
//   2. evaluates the residual of every admitted request (one launch per
//      (equation, dim, N+1, Nt) group) and its norm (one batched launch),
//   3. synchronises once, reads every request's state header, retires the
//      converged / failed / cancelled ones (u_next copied to the host), and
//   4. enqueues one GMRES cycle for the rest: per Arnoldi step one JVP launch
//      per (group, precision) and batched multi-dot / update / normalise
//      launches over all of them, then the Newton update.
// Requests of the scalar equations may ask for the element-block Jacobi
// preconditioner (right preconditioning, as in st_solve_slab): the block
// inverse is assembled on the submitting thread, uploaded at admission, and
// applied per Arnoldi step by one launch per block size.
// Requests that arrive while a tick runs are admitted at the next tick.  The
// per-request arithmetic is the single-slab driver's, with reductions that
// depend only on the request's own size, so results are bitwise independent
// of the batch.
#include "st_engine.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace stdg;

namespace {

constexpr int64_t ALIGN = 256;

int64_t align_up(int64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// First-fit allocator over one device arena (offsets), coalescing on free.
struct Arena {
    char* base = nullptr;
    int64_t size = 0;
    std::map<int64_t, int64_t> free_;   // offset -> length
    void init(char* b, int64_t n) {
        base = b;
        size = n;
        free_.clear();
        free_[0] = n;
    }
    char* alloc(int64_t n) {
        n = align_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                return base + off;
            }
        }
        return nullptr;
    }
    void release(char* p, int64_t n) {
        n = align_up(n);
        int64_t off = p - base;
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
};

struct Layout {
    int64_t U, R, w, V, uprev, unext, Q, dQ, U32, dQ32, part, pz, binv, total;
};

Layout layout_of(const Problem& pb, const st_solver_opts_t& o) {
    Layout L;
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t at = off; off += align_up(std::max<int64_t>(bytes, 8)); return at; };
    const int64_t n = pb.n;
    const bool visc = grad_pass(pb), nonlin = !linear_eq(pb.eq.kind), fp32 = o.inner_fp32 != 0;
    L.U = take(8 * n);
    L.R = take(8 * n);
    L.w = take(8 * n);
    L.V = take(8 * n * o.restart);
    L.uprev = take(8 * pb.nsp);
    L.unext = take(8 * pb.nsp);
    L.Q = visc ? take(8 * visc_len(pb)) : -1;
    L.dQ = visc ? take(8 * visc_len(pb)) : -1;
    L.U32 = (fp32 && nonlin) ? take(4 * n) : -1;
    L.dQ32 = (fp32 && visc) ? take(4 * visc_len(pb)) : -1;
    L.part = take(8 * (int64_t)vec_blocks(n) * (NPART_SLOTS + 1));
    // element-block Jacobi: the preconditioned direction and B^-1 (packed)
    const int npe = pb.nv * pb.Nt * pb.ns;
    const int64_t pk = (int64_t)((npe + 15) / 16) * ((npe + 3) / 4) * 64;
    L.pz = o.precond == 1 ? take(8 * n) : -1;
    L.binv = o.precond == 1 ? take(8 * pk) : -1;
    L.total = off;
    return L;
}

int check_opts(const st_solver_opts_t& o) {
    if (o.restart < 1 || o.restart > MMAX) return set_error(ST_ERR_BAD_ARG, "restart must be in 1..32");
    if (o.cgs_passes < 0 || o.cgs_passes > 2) return set_error(ST_ERR_BAD_ARG, "cgs_passes must be 0, 1 or 2");
    if (o.max_newton < 1) return set_error(ST_ERR_BAD_ARG, "max_newton must be >= 1");
    if (o.precond < 0 || o.precond > 1) return set_error(ST_ERR_BAD_ARG, "precond must be 0 or 1");
    return ST_OK;
}

enum Phase { QUEUED, ACTIVE, FINISHED };

struct Req {
    uint64_t ticket;
    Problem pb;
    st_solver_opts_t opts;
    double t0, dt, tol;
    std::vector<double> uprev;
    std::vector<double> unext;
    std::vector<double> binv;     // element-block Jacobi: B^-1 packed (until admitted)
    Layout lay;
    Phase phase = QUEUED;
    std::atomic<bool> cancel{false};
    bool fresh = true;
    int status = ST_PENDING;
    int slot = -1;
    char* mem = nullptr;
    int outer = 0;
    double r0 = 0.0, rn = 0.0, best = INFINITY;
    int stall = 0;
    double eta_rel = 0.0;
    st_stats_t stats{};
    double t_submit = 0, t_admit = 0, t_done = 0;

    double* dp(int64_t off) const { return off < 0 ? nullptr : (double*)(mem + off); }
    float* fp(int64_t off) const { return off < 0 ? nullptr : (float*)(mem + off); }
    bool fp32() const { return opts.inner_fp32 != 0; }
    bool pc() const { return opts.precond == 1; }
    int npe() const { return pb.nv * pb.Nt * pb.ns; }
};

}  // namespace

struct st_srv {
    st_server_opts_t opts;
    hipStream_t stream = nullptr;
    std::thread thr;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<Req*> queue;
    std::vector<Req*> active;
    std::unordered_map<uint64_t, Req*> all;
    uint64_t next_ticket = 1;
    int64_t bytes_in_use = 0;
    int64_t completed = 0, ticks = 0;
    Arena arena;
    char* d_arena = nullptr;
    GState* d_states = nullptr;   // one per slot
    GState* h_states = nullptr;   // pinned mirror (headers)
    std::vector<int> free_slots;
    // descriptor staging: two regions (residual phase, GMRES phase), pinned and device
    char* h_stage[2] = {nullptr, nullptr};
    char* d_stage[2] = {nullptr, nullptr};
    int64_t stage_cap = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now_us() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Descriptor tables of one launch phase, packed into a staging region.
struct Packer {
    std::vector<char> buf;
    template <class T>
    int64_t add(const std::vector<T>& v) {
        int64_t off = align_up((int64_t)buf.size());
        buf.resize(off + sizeof(T) * v.size());
        if (!v.empty()) std::memcpy(buf.data() + off, v.data(), sizeof(T) * v.size());
        return off;
    }
};

int upload(st_srv* s, int region, const Packer& pk) {
    const int64_t need = (int64_t)pk.buf.size();
    if (need > s->stage_cap) {
        int64_t cap = std::max<int64_t>(need * 2, 1 << 20);
        for (int r = 0; r < 2; ++r) {
            if (s->h_stage[r]) (void)hipHostFree(s->h_stage[r]);
            if (s->d_stage[r]) (void)hipFree(s->d_stage[r]);
            s->h_stage[r] = nullptr;
            s->d_stage[r] = nullptr;
            if (hipHostMalloc((void**)&s->h_stage[r], cap, hipHostMallocDefault) != hipSuccess ||
                hipMalloc((void**)&s->d_stage[r], cap) != hipSuccess)
                return ST_ERR_HIP;
        }
        s->stage_cap = cap;
    }
    if (need == 0) return ST_OK;
    std::memcpy(s->h_stage[region], pk.buf.data(), need);
    if (hipMemcpyAsync(s->d_stage[region], s->h_stage[region], need, hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return ST_ERR_HIP;
    return ST_OK;
}

VecSeg vecseg_of(st_srv* s, Req* r) {
    VecSeg v;
    std::memset(&v, 0, sizeof(v));
    v.V = r->dp(r->lay.V);
    v.w = r->dp(r->lay.w);
    v.R = r->dp(r->lay.R);
    v.U = r->dp(r->lay.U);
    v.n = r->pb.n;
    v.st = s->d_states + r->slot;
    v.part = r->dp(r->lay.part);
    v.part2 = v.part + (int64_t)vec_blocks(r->pb.n) * NPART_SLOTS;
    v.eta_rel = r->eta_rel;
    v.eta_tgt = 0.5;
    v.tol = r->tol;
    v.m = r->opts.restart;
    v.uprev = r->dp(r->lay.uprev);
    v.unext = r->dp(r->lay.unext);
    v.U32 = r->fp(r->lay.U32);
    v.nt = r->pb.Nt;
    v.ns = r->pb.ns;
    v.nblk = vec_blocks(r->pb.n);
    return v;
}

// Assign blk0 offsets; returns the total block count.
template <class Seg>
int assign_blocks(std::vector<Seg>& v) {
    int b = 0;
    for (auto& s : v) {
        s.blk0 = b;
        b += s.nblk;
    }
    return b;
}

struct OpGroup {
    const OpTable* ops;
    bool fp32;
    std::vector<OpSeg> grad, op;
    int64_t off_grad = 0, off_op = 0;
    int G = 0;
};

// Group key: operator table and precision.
std::vector<OpGroup> build_res_groups(st_srv* s, const std::vector<Req*>& rs) {
    std::vector<OpGroup> gs;
    for (Req* r : rs) {
        const Problem& pb = r->pb;
        OpGroup* g = nullptr;
        for (auto& x : gs)
            if (x.ops == pb.ops) g = &x;
        if (!g) {
            gs.push_back(OpGroup{pb.ops, false, {}, {}, 0, 0, 0});
            g = &gs.back();
        }
        OpSeg base = base_opseg(pb, r->dt);
        if (grad_pass(pb)) {
            OpSeg gr = base;
            visc_tiles(gr, pb);
            gr.U = dptr(r->dp(r->lay.U));
            gr.out = dptr(r->dp(r->lay.Q));
            g->grad.push_back(gr);
            base.Q = dptr(r->dp(r->lay.Q));
        }
        base.U = dptr(r->dp(r->lay.U));
        base.uprev = r->dp(r->lay.uprev);
        base.out = dptr(r->dp(r->lay.R));
        g->op.push_back(base);
    }
    (void)s;
    for (auto& g : gs) {
        g.G = assign_blocks(g.op);
        assign_blocks(g.grad);
    }
    return gs;
}

// JVP groups: the direction follows each request's device Arnoldi index.
std::vector<OpGroup> build_jvp_groups(st_srv* s, const std::vector<Req*>& rs) {
    std::vector<OpGroup> gs;
    for (Req* r : rs) {
        const Problem& pb = r->pb;
        const bool f32 = r->fp32();
        OpGroup* g = nullptr;
        for (auto& x : gs)
            if (x.ops == pb.ops && x.fp32 == f32) g = &x;
        if (!g) {
            gs.push_back(OpGroup{pb.ops, f32, {}, {}, 0, 0, 0});
            g = &gs.back();
        }
        GState* st = s->d_states + r->slot;
        // the direction: V_k (following the device Arnoldi index), or with
        // right preconditioning z = B^-1 V_k, formed before the launch
        DynPtr Vk = r->pc() ? dptr(r->dp(r->lay.pz)) : dptr_k(r->dp(r->lay.V), pb.n, &st->k);
        OpSeg b = base_opseg(pb, r->dt);
        b.skip = &st->done;
        b.out = dptr(r->dp(r->lay.w));
        const int kind = pb.eq.kind;
        void* dQ = f32 ? (void*)r->fp(r->lay.dQ32) : (void*)r->dp(r->lay.dQ);
        const DynPtr state = dptr(f32 ? (const void*)r->fp(r->lay.U32) : (const void*)r->dp(r->lay.U));
        if (grad_pass(pb)) {
            // NS viscous pass: tangent of -Fv at (U, v)
            OpSeg gr = b;
            visc_tiles(gr, pb);
            gr.U = state;
            gr.V = Vk;
            gr.out = dptr(dQ);
            g->grad.push_back(gr);
        }
        if (linear_eq(kind)) {
            b.U = Vk;
            b.uprev = nullptr;
            b.bcg = 0.0;
        } else {
            b.U = state;
            b.V = Vk;
            if (grad_pass(pb)) b.Q = dptr(dQ);
        }
        g->op.push_back(b);
    }
    for (auto& g : gs) {
        g.G = assign_blocks(g.op);
        assign_blocks(g.grad);
    }
    return gs;
}

void finish_request(st_srv* s, Req* r, int status) {
    r->status = status;
    r->phase = FINISHED;
    r->t_done = s->now_us();
    r->stats.newton_its = r->outer;
    r->stats.res0 = r->r0;
    r->stats.res_final = r->rn;
    r->stats.status = status;
    r->stats.usec = r->t_done - r->t_admit;
    if (r->mem) {
        s->arena.release(r->mem, r->lay.total);
        s->bytes_in_use -= align_up(r->lay.total);
        r->mem = nullptr;
    }
    if (r->slot >= 0) {
        s->free_slots.push_back(r->slot);
        r->slot = -1;
    }
    s->completed += 1;
}

// One scheduler tick; returns false when idle.
bool tick(st_srv* s) {
    std::vector<Req*> fresh;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // cancellations of queued requests
        for (auto it = s->queue.begin(); it != s->queue.end();) {
            if ((*it)->cancel) {
                finish_request(s, *it, ST_ERR_CANCELLED);
                it = s->queue.erase(it);
            } else {
                ++it;
            }
        }
        // admission (FIFO; a request that does not fit waits at the head)
        while (!s->queue.empty() && !s->free_slots.empty()) {
            Req* r = s->queue.front();
            char* mem = s->arena.alloc(r->lay.total);
            if (!mem) break;
            s->queue.pop_front();
            r->mem = mem;
            r->slot = s->free_slots.back();
            s->free_slots.pop_back();
            s->bytes_in_use += align_up(r->lay.total);
            r->phase = ACTIVE;
            r->t_admit = s->now_us();
            s->active.push_back(r);
            fresh.push_back(r);
        }
    }
    if (s->active.empty()) return false;
    s->ticks += 1;
    hipStream_t st = s->stream;

    // new requests: u_prev (and B^-1) upload, state reset, initial guess
    for (Req* r : fresh) {
        (void)hipMemcpyAsync(r->dp(r->lay.uprev), r->uprev.data(), 8 * r->pb.nsp, hipMemcpyHostToDevice, st);
        if (r->pc())
            (void)hipMemcpyAsync(r->dp(r->lay.binv), r->binv.data(), 8 * r->binv.size(), hipMemcpyHostToDevice, st);
        (void)hipMemsetAsync(s->d_states + r->slot, 0, sizeof(GState), st);
    }
    // phase A: residual and norm of every active request
    Packer pa;
    std::vector<VecSeg> vall;
    for (Req* r : s->active) vall.push_back(vecseg_of(s, r));
    const int Gall = assign_blocks(vall);
    std::vector<VecSeg> vfresh;
    for (Req* r : fresh) vfresh.push_back(vecseg_of(s, r));
    const int Gfresh = assign_blocks(vfresh);
    auto rgroups = build_res_groups(s, s->active);
    const int64_t off_vall = pa.add(vall), off_vfresh = pa.add(vfresh);
    for (auto& g : rgroups) {
        g.off_grad = pa.add(g.grad);
        g.off_op = pa.add(g.op);
    }
    if (upload(s, 0, pa) != ST_OK) return true;
    char* D0 = s->d_stage[0];
    if (!vfresh.empty()) vk_init_guess((VecSeg*)(D0 + off_vfresh), (int)vfresh.size(), Gfresh, st);
    for (auto& g : rgroups) {
        if (!g.grad.empty()) g.ops->visc_res64((OpSeg*)(D0 + g.off_grad), (int)g.grad.size(), g.G, st);
        g.ops->res64((OpSeg*)(D0 + g.off_op), (int)g.op.size(), g.G, st);
    }
    vk_rnorm((VecSeg*)(D0 + off_vall), (int)vall.size(), Gall, st);
    vk_begin((VecSeg*)(D0 + off_vall), (int)vall.size(), st);
    // headers of every slot's state
    const size_t hdr = offsetof(GState, hacc);
    (void)hipMemcpy2DAsync(s->h_states, sizeof(GState), s->d_states, sizeof(GState), hdr, s->opts.max_active,
                           hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Req* r : s->active) finish_request(s, r, ST_ERR_HIP);
        s->active.clear();
        return true;
    }

    // decisions
    std::vector<Req*> cont, retire;
    for (Req* r : s->active) {
        const GState& hs = s->h_states[r->slot];
        r->rn = hs.rnorm;
        if (r->fresh) { r->r0 = r->rn; r->fresh = false; }
        r->stats.gmres_its = hs.iters_total;
        int status = ST_PENDING;
        if (r->cancel) status = ST_ERR_CANCELLED;
        else if (hs.nonfinite) status = ST_ERR_NONFINITE;
        else if (r->rn <= hs.target) status = ST_OK;
        else if (r->outer >= r->opts.max_newton) status = ST_ERR_NO_CONVERGENCE;
        else if (r->rn < 0.9 * r->best) { r->best = r->rn; r->stall = 0; }
        else if (++r->stall >= 8) status = ST_ERR_NO_CONVERGENCE;
        if (status == ST_PENDING) { r->outer += 1; cont.push_back(r); }
        else { r->status = status; retire.push_back(r); }
    }
    if (!retire.empty()) {
        std::vector<VecSeg> vr;
        for (Req* r : retire) vr.push_back(vecseg_of(s, r));
        const int Gr = assign_blocks(vr);
        Packer pr;
        const int64_t off = pr.add(vr);
        if (upload(s, 1, pr) == ST_OK) {
            vk_extract_last((VecSeg*)(s->d_stage[1] + off), (int)vr.size(), Gr, st);
            for (Req* r : retire) {
                r->unext.resize(r->pb.nsp);
                (void)hipMemcpyAsync(r->unext.data(), r->dp(r->lay.unext), 8 * r->pb.nsp, hipMemcpyDeviceToHost, st);
            }
            (void)hipStreamSynchronize(st);
        }
        std::lock_guard<std::mutex> lk(s->mu);
        for (Req* r : retire) {
            finish_request(s, r, r->status);
            s->active.erase(std::find(s->active.begin(), s->active.end(), r));
        }
    }
    if (cont.empty()) return true;

    // phase B: one GMRES cycle and the Newton update for every continuing request
    Packer pb;
    std::vector<VecSeg> vc;
    for (Req* r : cont) vc.push_back(vecseg_of(s, r));
    const int Gc = assign_blocks(vc);
    const int64_t off_vc = pb.add(vc);
    // the Gram-Schmidt launches by form ([0] CGS, [1] CGS2, [2] adaptive), so
    // that a request gets its own passes whatever it is batched with
    std::vector<VecSeg> vp[3];
    for (Req* r : cont) vp[r->opts.cgs_passes == 0 ? 2 : r->opts.cgs_passes - 1].push_back(vecseg_of(s, r));
    int Gp[3];
    int64_t off_vp[3];
    for (int q = 0; q < 3; ++q) {
        Gp[q] = assign_blocks(vp[q]);
        off_vp[q] = pb.add(vp[q]);
    }
    std::vector<Req*> c32;
    for (Req* r : cont)
        if (r->fp32() && !linear_eq(r->pb.eq.kind)) c32.push_back(r);
    std::vector<VecSeg> v32;
    for (Req* r : c32) v32.push_back(vecseg_of(s, r));
    const int G32 = assign_blocks(v32);
    const int64_t off_v32 = pb.add(v32);
    auto jgroups = build_jvp_groups(s, cont);
    for (auto& g : jgroups) {
        g.off_grad = pb.add(g.grad);
        g.off_op = pb.add(g.op);
    }
    // element-block Jacobi: z = B^-1 V_k before each JVP and U += B^-1 (V y)
    // at the end, one launch per block size; the Newton update of the other
    // requests stays U += V y
    struct PcGroup {
        int npe;
        std::vector<PcSeg> step, upd;
        int64_t off_step = 0, off_upd = 0;
        int G = 0;
    };
    std::vector<PcGroup> pgroups;
    std::vector<VecSeg> vpc, vplain;
    for (Req* r : cont) {
        if (!r->pc()) {
            vplain.push_back(vecseg_of(s, r));
            continue;
        }
        vpc.push_back(vecseg_of(s, r));
        PcGroup* g = nullptr;
        for (auto& x : pgroups)
            if (x.npe == r->npe()) g = &x;
        if (!g) {
            pgroups.push_back(PcGroup{r->npe(), {}, {}, 0, 0, 0});
            g = &pgroups.back();
        }
        GState* gs = s->d_states + r->slot;
        PcSeg a;
        std::memset(&a, 0, sizeof(a));
        a.in = dptr_k(r->dp(r->lay.V), r->pb.n, &gs->k);
        a.out = r->dp(r->lay.pz);
        a.binvT = r->dp(r->lay.binv);
        a.skip = &gs->done;
        a.npe = r->npe();
        a.E = (int)r->pb.E;
        a.accumulate = 0;
        a.nblk = pc_blocks(a.E, a.npe);
        g->step.push_back(a);
        PcSeg u = a;
        u.in = dptr(r->dp(r->lay.w));
        u.out = r->dp(r->lay.U);
        u.skip = nullptr;
        u.accumulate = 1;
        g->upd.push_back(u);
    }
    for (auto& g : pgroups) {
        g.G = assign_blocks(g.step);
        assign_blocks(g.upd);
        g.off_step = pb.add(g.step);
        g.off_upd = pb.add(g.upd);
    }
    const int Gpc = assign_blocks(vpc), Gplain = assign_blocks(vplain);
    const int64_t off_vpc = pb.add(vpc), off_vplain = pb.add(vplain);
    if (upload(s, 1, pb) != ST_OK) return true;
    char* D1 = s->d_stage[1];
    if (!v32.empty()) vk_cast32((VecSeg*)(D1 + off_v32), (int)v32.size(), G32, st);
    VecSeg* dvc = (VecSeg*)(D1 + off_vc);
    const int nc = (int)vc.size();
    int mmax = 0;
    int64_t basis = 0;                    // Krylov bases of the tick's requests, bytes
    for (Req* r : cont) {
        mmax = std::max(mmax, r->opts.restart);
        basis += (int64_t)(r->opts.restart + 1) * r->pb.n * 8;
    }
    const int gstream = gs_stream(basis);
    vk_scale_v0(dvc, nc, Gc, st);
    for (int k = 0; k < mmax; ++k) {
        for (auto& g : pgroups) pc_apply((PcSeg*)(D1 + g.off_step), (int)g.step.size(), g.G, g.npe, st);
        for (auto& g : jgroups) {
            if (!g.grad.empty())
                (g.fp32 ? g.ops->visc_jvp32 : g.ops->visc_jvp64)((OpSeg*)(D1 + g.off_grad), (int)g.grad.size(), g.G, st);
            OpLaunch f = linear_eq(g.ops->eq) ? (g.fp32 ? g.ops->lin32 : g.ops->res64)
                                              : (g.fp32 ? g.ops->jvp32 : g.ops->jvp64);
            f((OpSeg*)(D1 + g.off_op), (int)g.op.size(), g.G, st);
        }
        for (int q = 0; q < 3; ++q) {
            if (vp[q].empty()) continue;
            VecSeg* dq = (VecSeg*)(D1 + off_vp[q]);
            const int nq = (int)vp[q].size();
            const int passes = q == 2 ? 0 : q + 1;
            for (int p = 0; p < (q == 0 ? 1 : 2); ++p) {
                int lastp = 0, gate = 0;
                gs_pass_plan(passes, p, &lastp, &gate);
                vk_multidot(dq, nq, Gp[q], k, st, gate, gstream);
                vk_update(dq, nq, Gp[q], p, lastp, k, st, gstream);
            }
        }
    }
    vk_finish(dvc, nc, st);
    if (!vplain.empty()) vk_update_u((VecSeg*)(D1 + off_vplain), (int)vplain.size(), Gplain, st);
    if (!vpc.empty()) {
        pc_combine((VecSeg*)(D1 + off_vpc), (int)vpc.size(), Gpc, st);
        for (auto& g : pgroups) pc_apply((PcSeg*)(D1 + g.off_upd), (int)g.upd.size(), g.G, g.npe, st);
    }
    return true;
}

void scheduler(st_srv* s) {
    (void)hipSetDevice(s->opts.device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop) break;
            if (s->active.empty() && s->queue.empty()) {
                s->cv.wait_for(lk, std::chrono::milliseconds(50));
                continue;
            }
        }
        tick(s);
    }
}

}  // namespace

extern "C" {

int64_t st_request_footprint(const st_request_t* req) {
    if (!req) return -1;
    Problem pb;
    if (make_problem(&req->mesh, req->N, req->Nt, &req->eq, pb) != ST_OK) return -1;
    return align_up(layout_of(pb, req->opts).total);
}

int st_server_create(const st_server_opts_t* opts, st_server_t* out) {
    if (!opts || !out) return set_error(ST_ERR_BAD_ARG, "null argument");
    if (opts->max_active < 1 || opts->hbm_budget_bytes < (1 << 20))
        return set_error(ST_ERR_BAD_ARG, "need max_active >= 1 and a budget of at least 1 MiB");
    st_srv* s = new st_srv();
    s->opts = *opts;
    if (hipSetDevice(opts->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void**)&s->d_arena, opts->hbm_budget_bytes) != hipSuccess ||
        hipMalloc((void**)&s->d_states, sizeof(GState) * opts->max_active) != hipSuccess ||
        hipHostMalloc((void**)&s->h_states, sizeof(GState) * opts->max_active, hipHostMallocDefault) != hipSuccess) {
        st_server_destroy(s);
        return set_error(ST_ERR_HIP, "server allocation failed");
    }
    s->arena.init(s->d_arena, opts->hbm_budget_bytes);
    for (int i = opts->max_active - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->thr = std::thread(scheduler, s);
    *out = s;
    return ST_OK;
}

int st_server_destroy(st_server_t s) {
    if (!s) return set_error(ST_ERR_BAD_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->thr.joinable()) s->thr.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->all) delete kv.second;
    for (int r = 0; r < 2; ++r) {
        if (s->h_stage[r]) (void)hipHostFree(s->h_stage[r]);
        if (s->d_stage[r]) (void)hipFree(s->d_stage[r]);
    }
    if (s->h_states) (void)hipHostFree(s->h_states);
    if (s->d_states) (void)hipFree(s->d_states);
    if (s->d_arena) (void)hipFree(s->d_arena);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return ST_OK;
}

int st_submit(st_server_t s, const st_request_t* req, uint64_t* ticket) {
    if (!s || !req || !ticket || !req->u_prev) return set_error(ST_ERR_BAD_ARG, "null argument");
    if (!(req->dt > 0.0) || !(req->tol > 0.0)) return set_error(ST_ERR_BAD_ARG, "dt and tol must be positive");
    Req* r = new Req();
    int rc = make_problem(&req->mesh, req->N, req->Nt, &req->eq, r->pb);
    if (rc == ST_OK) rc = check_opts(req->opts);
    if (rc != ST_OK) { delete r; return rc; }
    r->opts = req->opts;
    r->t0 = req->t0;
    r->dt = req->dt;
    r->tol = req->tol;
    r->lay = layout_of(r->pb, r->opts);
    if (align_up(r->lay.total) > s->opts.hbm_budget_bytes) {
        int64_t need = r->lay.total;
        delete r;
        return set_error(ST_ERR_OOM_ADMISSION, "request needs " + std::to_string(need) + " bytes, budget is " +
                                                   std::to_string(s->opts.hbm_budget_bytes));
    }
    r->eta_rel = linear_eq(r->pb.eq.kind) ? 0.0 : std::max(r->opts.gmres_rtol, 0.0);
    if (r->fp32()) r->eta_rel = std::max(r->eta_rel, 1e-5);
    r->uprev.assign(req->u_prev, req->u_prev + r->pb.nsp);
    if (r->pc()) {
        // element-block Jacobi: scalar equations only (their block is
        // assembled on the host, here, on the submitting thread)
        if (r->pb.nv != 1) rc = set_error(ST_ERR_UNSUPPORTED, "served preconditioning: scalar equations only");
        if (rc == ST_OK) rc = scalar_block_inverse(r->pb, r->uprev.data(), r->dt, r->binv);
        if (rc == ST_OK && pc_prepare(r->npe()) != hipSuccess)
            rc = set_error(ST_ERR_UNSUPPORTED, "element block needs more LDS than the device grants");
        if (rc != ST_OK) { delete r; return rc; }
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        r->t_submit = s->now_us();
        s->all[r->ticket] = r;
        s->queue.push_back(r);
    }
    s->cv.notify_all();
    *ticket = r->ticket;
    return ST_OK;
}

int st_poll(st_server_t s, uint64_t ticket, st_result_t* out) {
    if (!s) return set_error(ST_ERR_BAD_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(ST_ERR_NOT_FOUND, "unknown ticket " + std::to_string(ticket));
    Req* r = it->second;
    if (r->phase != FINISHED) return ST_PENDING;
    if (out) {
        out->status = r->status;
        if (out->u_next && !r->unext.empty()) std::memcpy(out->u_next, r->unext.data(), 8 * r->unext.size());
        out->stats = r->stats;
        out->submit_us = r->t_submit;
        out->admit_us = r->t_admit;
        out->done_us = r->t_done;
    }
    const int status = r->status;
    s->all.erase(it);
    delete r;
    return status;
}

int st_cancel(st_server_t s, uint64_t ticket) {
    if (!s) return set_error(ST_ERR_BAD_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(ST_ERR_NOT_FOUND, "unknown ticket " + std::to_string(ticket));
    it->second->cancel = true;
    s->cv.notify_all();
    return ST_OK;
}

int st_server_stats(st_server_t s, int64_t* queued, int64_t* active, int64_t* completed, int64_t* ticks,
                    int64_t* bytes_in_use) {
    if (!s) return set_error(ST_ERR_BAD_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int64_t)s->queue.size();
    if (active) *active = (int64_t)s->active.size();
    if (completed) *completed = s->completed;
    if (ticks) *ticks = s->ticks;
    if (bytes_in_use) *bytes_in_use = s->bytes_in_use;
    return ST_OK;
}

}  // extern "C"
