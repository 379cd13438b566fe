// Batched solves: many right-hand sides on each of many lattices of uneven size.
//
// One host thread drives all lattices.  Per lattice (one context) every kernel of a GCR iteration
// covers all of its right-hand sides in one launch, with per-system scalars and an active mask that
// freezes converged systems.  The launch sequence of iteration k of a cycle, for all lattices at
// once (one branch per lattice, so the lattices run concurrently), is captured into one hipGraph
// and replayed: one graph launch per iteration for the whole batch.  Convergence is decided on the
// device: after each iteration a small kernel per lattice compares each active system's residual
// norm with its target, clears the system's mask entry, counts its iterations and the systems still
// active; a last node gathers the counts of all lattices into one array, which the host reads only
// every kPoll iterations and at the end of a cycle.  The end of a cycle (back-substitution, solution
// update, true residual, restart decision) is device work too, in one graph per cycle length.
// Method: FP64 even-odd GCR, or FP64 defect correction around a batched inner GCR in
// FP32 / FP16 / BF16 (the mixed scheme of solver.hip, per system).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "blas.h"

namespace dl {

namespace {
std::atomic<unsigned long long> g_bwork_ids{1};
}

struct BWork {
    unsigned long long id = g_bwork_ids++;  // identifies this work space in graph keys
    hipStream_t s = nullptr;                // the lattice's stream (set-up and per-lattice steps)
    DevBuf P, Q, r, e, b, act, cyc, cnt;
    DevBuf stage;                   // device staging of per-system values (contiguous)
    unsigned char *pin = nullptr;   // pinned host staging (kPinBytes): every host <-> device value copy
    DevBuf h64[4];  // FP64 half vectors x nrhs: eta-hat, x_e, r, tmp
    DevBuf f64[3];  // FP64 full vectors x nrhs: b, x, r
    // batch-level state, used when this lattice leads a batch (is its first lattice)
    hipStream_t ms = nullptr;  // the batch stream: graphs and the GCR cycles of all lattices
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> ev;  // one per lattice: branch joins and stream hand-overs
    DevBuf table, nact;          // device pointers to every lattice's active count; gathered counts
    int *host_nact = nullptr;    // pinned copy of the gathered counts
    int nlat_cap = 0;
    std::vector<hipGraphExec_t> it_graphs, end_graphs;
    hipGraphExec_t start_graph = nullptr;
    std::vector<unsigned long long> graph_key;
    void drop_graphs() {
        for (auto g : it_graphs)
            if (g) (void)hipGraphExecDestroy(g);
        for (auto g : end_graphs)
            if (g) (void)hipGraphExecDestroy(g);
        if (start_graph) (void)hipGraphExecDestroy(start_graph);
        it_graphs.clear();
        end_graphs.clear();
        start_graph = nullptr;
        graph_key.clear();
    }
    ~BWork() {
        drop_graphs();
        if (s) (void)hipStreamDestroy(s);
        if (ms) (void)hipStreamDestroy(ms);
        if (fork) (void)hipEventDestroy(fork);
        for (auto e : ev) (void)hipEventDestroy(e);
        if (host_nact) (void)hipHostFree(host_nact);
        if (pin) (void)hipHostFree(pin);
        for (DevBuf *d : {&P, &Q, &r, &e, &b, &act, &cyc, &cnt, &table, &nact, &stage}) d->release();
        for (auto &d : h64) d.release();
        for (auto &d : f64) d.release();
    }
};

namespace {

constexpr int S_RED = 0, S_SC = 8, S_MISC = 16, S_GAM = 64, S_ALP = 192, S_C = 320, S_BETA = 512;
constexpr int S_ALPHA = kSysScal - 64, S_XS = kSysScal - 62, S_ONE = kSysScal - 60;  // per-system free slots
constexpr int S_TGT = kSysScal - 56;  // per-system target of the current GCR (normalised norm)
constexpr int kMaxM = 64;
constexpr int kPoll = 4;  // iterations between two host reads of the active counts

bool graphs_enabled() {
    const char *e = getenv("DIRAC_GRAPHS");
    return !e || atoi(e) != 0;
}

// ------------------------------------------------------------------ device-side GCR control
// Per-system counters of a lattice (int, R systems): [0, R) iterations, [R, 2R) restarts,
// [2R, 3R) iterations in the current cycle, [3R, 4R) flags (1 converged, 2 non-finite),
// [4R] systems still active.

// mode 0: after iteration k of a cycle (the systems in act); 1: start of a solve (the systems in
// act); 2: end of a cycle, after the true residual (the systems in cyc).  A system whose residual
// norm is not finite, or at most its target, leaves the active set; at the start and the end of a
// cycle the latter is marked converged, and at the end of a cycle the others restart.  One
// wavefront; the count of active systems is summed in a fixed order.
__global__ void k_bat_status(int R, int mode, int k, int *act, const int *cyc, int *cnt, const double *scal) {
    __shared__ int part[64];
    int na = 0;
    for (int q = threadIdx.x; q < R; q += 64) {
        const bool in = mode == 2 ? cyc[q] != 0 : act[q] != 0;
        if (in) {
            const double *sq = scal + (size_t)q * kSysScal;
            const double rn2 = sq[S_RED + 4];
            if (mode == 0) {
                ++cnt[q];
                cnt[2 * R + q] = k + 1;
            }
            if (!isfinite(rn2)) {
                cnt[3 * R + q] |= 2;
                act[q] = 0;
            } else if (sqrt(rn2) <= sq[S_TGT]) {
                act[q] = 0;
                if (mode != 0) cnt[3 * R + q] |= 1;
            } else if (mode == 2) {
                act[q] = 1;
                ++cnt[R + q];
            }
        }
        na += act[q] != 0;
    }
    part[threadIdx.x] = na;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int j = 0; j < 64; ++j) s += part[j];
        cnt[4 * R] = s;
    }
}

// Start of a cycle: the cycle's systems are the active ones; their cycle lengths restart at 0.
__global__ void k_bat_cycle_start(int R, const int *act, int *cyc, int *cnt) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= R) return;
    cyc[q] = act[q];
    cnt[2 * R + q] = 0;
}

// GCR back-substitution per system of the cycle over its own cycle length n:
// alpha_j = c_j gamma_j + sum_{k > j} c_k beta_jk, solved for c_{n-1} .. c_0; c_j = 0 for n <= j < kmax.
__global__ void k_bat_backsub(int R, const int *cyc, const int *cnt, double *scal, int kmax) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= R || !cyc[q]) return;
    double *b = scal + (size_t)q * kSysScal;
    const int n = cnt[2 * R + q];
    for (int j = kmax - 1; j >= n; --j) {
        b[S_C + 2 * j] = 0.0;
        b[S_C + 2 * j + 1] = 0.0;
    }
    for (int j = n - 1; j >= 0; --j) {
        double ar = b[S_ALP + 2 * j], ai = b[S_ALP + 2 * j + 1];
        for (int k = j + 1; k < n; ++k) {
            const double br = b[S_BETA + 2 * kMaxM * k + 2 * j], bi = b[S_BETA + 2 * kMaxM * k + 2 * j + 1];
            const double cr = b[S_C + 2 * k], ci = b[S_C + 2 * k + 1];
            ar -= br * cr - bi * ci;
            ai -= br * ci + bi * cr;
        }
        const double g = b[S_GAM + j];
        b[S_C + 2 * j] = ar / g;
        b[S_C + 2 * j + 1] = ai / g;
    }
}

// dst[r] = src[r * stride] and back: per-system scalars to and from a contiguous staging array.
__global__ void k_sys_gather(int n, const double *src, int stride, double *dst) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) dst[r] = src[(size_t)r * stride];
}
__global__ void k_sys_scatter(int n, const double *src, double *dst, int stride) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) dst[(size_t)r * stride] = src[r];
}

// out[l] = *src[l]: the active counts of all lattices into one array.
__global__ void k_gather_counts(int n, const int *const *src, int *out) {
    const int l = threadIdx.x;
    if (l < n) out[l] = *src[l];
}

struct Lat {
    dirac_ctx *c;
    BWork *w;
    int nrhs;
    double *scal() { return (double *)c->work->blas.scal.p; }
    double *sp(int slot) { return scal() + slot; }
    BatchSpec spec(const int *act) const { return BatchSpec{nrhs, act, kSysScal}; }
    int *act() { return (int *)w->act.p; }
    int *cyc() { return (int *)w->cyc.p; }
    int *cnt() { return (int *)w->cnt.p; }
};

// Host <-> device values of a lattice go through its pinned staging memory: per-system scalars
// (strided by kSysScal on the device) are gathered into / scattered from a contiguous device array
// by a small kernel, so every copy is a plain 1-D copy between device and pinned memory.
// Pinned layout: ints at [0, kPinInts), doubles after them.
constexpr int kPinInts = 512, kPinDoubles = 256;
constexpr size_t kPinBytes = kPinInts * sizeof(int) + kPinDoubles * sizeof(double);
int *pin_ints(Lat &L) { return (int *)L.w->pin; }
double *pin_doubles(Lat &L) { return (double *)(L.w->pin + kPinInts * sizeof(int)); }

// queue: device per-system slot -> pinned doubles (no wait)
void gather_sys(Lat &L, int slot, hipStream_t s) {
    k_sys_gather<<<1, 64, 0, s>>>(L.nrhs, L.sp(slot), kSysScal, (double *)L.w->stage.p);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(pin_doubles(L), L.w->stage.p, L.nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
}
// queue: pinned doubles -> device per-system slot (the pinned values must stay until s has run it)
void scatter_sys(Lat &L, int slot, hipStream_t s) {
    HIP_CHECK(hipMemcpyAsync(L.w->stage.p, pin_doubles(L), L.nrhs * sizeof(double), hipMemcpyHostToDevice, s));
    k_sys_scatter<<<1, 64, 0, s>>>(L.nrhs, (const double *)L.w->stage.p, L.sp(slot), kSysScal);
    HIP_CHECK(hipGetLastError());
}
// strided per-system scalars <-> host (on the lattice's stream, blocking)
void read_sys(Lat &L, int slot, std::vector<double> &h, hipStream_t s) {
    gather_sys(L, slot, s);
    HIP_CHECK(hipStreamSynchronize(s));
    h.assign(pin_doubles(L), pin_doubles(L) + L.nrhs);
}
void write_sys(Lat &L, int slot, const std::vector<double> &h, hipStream_t s) {
    std::copy(h.begin(), h.begin() + L.nrhs, pin_doubles(L));
    scatter_sys(L, slot, s);
    HIP_CHECK(hipStreamSynchronize(s));  // the pinned values are reused by the next call
}
void upload_mask(Lat &L, const std::vector<int> &m, int *d, hipStream_t s) {
    std::copy(m.begin(), m.begin() + L.nrhs, pin_ints(L));
    HIP_CHECK(hipMemcpyAsync(d, pin_ints(L), L.nrhs * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));  // idem
}

struct BOut {
    std::vector<int> iters, restarts;
    std::vector<char> converged;
    bool nonfinite = false;
};

// The batch: its lattices, the leader's batch-level state and the host reads it made.
struct Batch {
    std::vector<Lat> lats;
    BWork *lead = nullptr;
    long syncs = 0;  // host waits on the device during the solve
    bool concurrent = true;  // lattices as concurrent graph branches (else one after another)
    hipStream_t ms() const { return lead->ms; }
    // the batch stream waits for everything queued on the lattice streams, or the reverse
    void lattices_to_batch() {
        for (size_t l = 0; l < lats.size(); ++l) {
            HIP_CHECK(hipEventRecord(lead->ev[l], lats[l].w->s));
            HIP_CHECK(hipStreamWaitEvent(lead->ms, lead->ev[l], 0));
        }
    }
    void batch_to_lattices() {
        HIP_CHECK(hipEventRecord(lead->fork, lead->ms));
        for (auto &L : lats) HIP_CHECK(hipStreamWaitEvent(L.w->s, lead->fork, 0));
    }
    // Run body(l, stream) for every lattice on the batch stream: inside a capture, as concurrent
    // branches forked from and joined back into the batch stream; otherwise one after another.
    template <typename F>
    void branches(bool capture, F &&body) {
        if (!capture || !concurrent) {
            for (size_t l = 0; l < lats.size(); ++l) body((int)l, ms());
            return;
        }
        HIP_CHECK(hipEventRecord(lead->fork, ms()));
        for (size_t l = 0; l < lats.size(); ++l) {
            hipStream_t s = lats[l].w->s;
            HIP_CHECK(hipStreamWaitEvent(s, lead->fork, 0));
            body((int)l, s);
            HIP_CHECK(hipEventRecord(lead->ev[l], s));
            HIP_CHECK(hipStreamWaitEvent(ms(), lead->ev[l], 0));
        }
    }
    void gather(hipStream_t s) {
        k_gather_counts<<<1, 64, 0, s>>>((int)lats.size(), (const int *const *)lead->table.p, (int *)lead->nact.p);
        HIP_CHECK(hipGetLastError());
    }
    // total systems still active, read from the gathered counts (blocking)
    int poll() {
        HIP_CHECK(hipMemcpyAsync(lead->host_nact, lead->nact.p, lats.size() * sizeof(int), hipMemcpyDeviceToHost,
                                 ms()));
        HIP_CHECK(hipStreamSynchronize(ms()));
        ++syncs;
        int t = 0;
        for (size_t l = 0; l < lats.size(); ++l) t += lead->host_nact[l];
        return t;
    }
    // launch `record` as a graph held in `slot` (captured on first use), or directly
    template <typename F>
    void run_graph(bool use_graph, hipGraphExec_t &slot, F &&record) {
        if (!use_graph) {
            record(false);
            return;
        }
        if (!slot) {
            hipGraph_t g = nullptr;
            HIP_CHECK(hipStreamBeginCapture(ms(), hipStreamCaptureModeThreadLocal));
            try {
                record(true);
            } catch (...) {
                (void)hipStreamEndCapture(ms(), &g);  // leave the stream out of capture mode
                if (g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
                throw;
            }
            HIP_CHECK(hipStreamEndCapture(ms(), &g));
            HIP_CHECK(hipGraphInstantiate(&slot, g, nullptr, nullptr, 0));
            HIP_CHECK(hipGraphDestroy(g));
        }
        HIP_CHECK(hipGraphLaunch(slot, ms()));
    }
};

// Batched GCR(m) on D-hat for every lattice l in precision pr[l], for the systems with start = 1:
// x solves D-hat x = b to |b - D-hat x| <= target (normalised norms), x = 0 initially.  x[l], b[l]:
// nrhs half vectors of pr[l].  All work runs on the batch stream, ordered after the lattice streams.
std::vector<BOut> gcr_batched(Batch &B, const std::vector<dirac_prec> &pr, const std::vector<void *> &x,
                              const std::vector<const void *> &b, const std::vector<std::vector<int>> &start,
                              const std::vector<std::vector<double>> &target, int m, int max_iter, bool use_graph) {
    const int nl = (int)B.lats.size();
    hipStream_t ms = B.ms();
    B.lattices_to_batch();
    std::vector<unsigned long long> key = {(unsigned long long)m, (unsigned long long)nl};
    for (int l = 0; l < nl; ++l) {
        Lat &L = B.lats[l];
        dirac_ctx *c = L.c;
        const int R = L.nrhs;
        c->f[pr[l]].tmp_half.alloc((size_t)R * 24 * real_size(pr[l]) * c->g.vhp);
        std::copy(start[l].begin(), start[l].begin() + R, pin_ints(L));
        std::copy(target[l].begin(), target[l].begin() + R, pin_doubles(L));
        HIP_CHECK(hipMemcpyAsync(L.act(), pin_ints(L), R * sizeof(int), hipMemcpyHostToDevice, ms));
        HIP_CHECK(hipMemsetAsync(L.cnt(), 0, (4 * R + 1) * sizeof(int), ms));
        scatter_sys(L, S_TGT, ms);
        for (const unsigned long long v :
             {L.w->id, (unsigned long long)pr[l], (unsigned long long)R, (unsigned long long)(uintptr_t)x[l],
              (unsigned long long)(uintptr_t)b[l], (unsigned long long)(uintptr_t)c->work->blas.part.p,
              (unsigned long long)(uintptr_t)c->work->blas.scal.p,
              (unsigned long long)(uintptr_t)c->f[pr[l]].tmp_half.p, (unsigned long long)(uintptr_t)L.w->P.p,
              (unsigned long long)(uintptr_t)L.w->Q.p, (unsigned long long)(uintptr_t)L.w->r.p,
              (unsigned long long)(uintptr_t)L.w->act.p, (unsigned long long)(uintptr_t)L.w->cyc.p,
              (unsigned long long)(uintptr_t)L.w->cnt.p})
            key.push_back(v);
    }
    BWork &lw = *B.lead;
    if (use_graph && key != lw.graph_key) {
        lw.drop_graphs();
        lw.graph_key = key;
    }
    lw.it_graphs.resize(m, nullptr);
    lw.end_graphs.resize(m + 1, nullptr);
    auto blas = [&](int l) -> Blas & { return B.lats[l].c->work->blas; };
    auto scale = [&](int l) { return 1.0 / (24.0 * (double)B.lats[l].c->vh); };
    auto vbytes = [&](int l) { return (size_t)24 * real_size(pr[l]) * B.lats[l].c->g.vhp * B.lats[l].nrhs; };
    // x = 0, r = b, |r|, and the systems already converged leave
    for (int l = 0; l < nl; ++l) {
        Lat &L = B.lats[l];
        const int R = L.nrhs;
        blas(l).lincomb(pr[l], pr[l], pr[l], 1, x[l], nullptr, 0.0, b[l], 0.0, nullptr, nullptr, 1.0, ms,
                        L.spec(L.act()));
        blas(l).lincomb(pr[l], pr[l], pr[l], 1, L.w->r.p, nullptr, 1.0, b[l], 0.0, nullptr, L.sp(S_RED + 4),
                        scale(l), ms, L.spec(L.act()));
        k_bat_status<<<1, 64, 0, ms>>>(R, 1, 0, L.act(), L.cyc(), L.cnt(), L.scal());
        HIP_CHECK(hipGetLastError());
    }
    B.gather(ms);
    int active = B.poll();  // also completes the uploads above from the pinned staging
    // the launch-shape tuner cannot time candidates inside a capture: one eager operator
    // application per lattice (on the residual, into basis slot 0, which iteration 0 overwrites)
    // lets it choose before the graphs are recorded
    if (use_graph && !lw.it_graphs[0])
        for (int l = 0; l < nl; ++l)
            schur_apply(B.lats[l].c, B.lats[l].w->Q.p, B.lats[l].w->r.p, 0, pr[l], ms, B.lats[l].nrhs,
                        B.lats[l].act());
    auto iteration = [&](int l, int k, hipStream_t s) {
        Lat &L = B.lats[l];
        const size_t kb = vbytes(l);
        char *P = (char *)L.w->P.p, *Q = (char *)L.w->Q.p;
        char *qk = Q + k * kb;
        Blas &Bl = blas(l);
        const double sc = scale(l);
        schur_apply(L.c, qk, P + k * kb, 0, pr[l], s, L.nrhs, L.act());
        double *bcol = L.sp(S_BETA + 2 * kMaxM * k);
        if (k > 0) Bl.mdot(pr[l], 1, Q, k, qk, bcol, sc, s, L.spec(L.act()));
        Bl.maxpy_dot(pr[l], 1, Q, k, bcol, qk, L.w->r.p, L.sp(S_RED), sc, s, L.spec(L.act()));
        Bl.gcr_scalars(L.sp(S_RED), L.sp(S_SC), L.sp(S_GAM), L.sp(S_ALP), k, s, L.spec(L.act()));
        Bl.gcr_update(pr[l], 1, L.sp(S_SC), qk, L.w->r.p, P + (k + 1) * kb, L.sp(S_RED + 4), sc, s,
                      L.spec(L.act()));
        k_bat_status<<<1, 64, 0, s>>>(L.nrhs, 0, k, L.act(), L.cyc(), L.cnt(), L.scal());
        HIP_CHECK(hipGetLastError());
    };
    auto cycle_start = [&](int l, hipStream_t s) {
        Lat &L = B.lats[l];
        k_bat_cycle_start<<<1, 64, 0, s>>>(L.nrhs, L.act(), L.cyc(), L.cnt());
        HIP_CHECK(hipGetLastError());
        blas(l).lincomb(pr[l], pr[l], pr[l], 1, L.w->P.p, nullptr, 1.0, L.w->r.p, 0.0, nullptr, nullptr, 1.0, s,
                        L.spec(L.act()));
    };
    auto cycle_end = [&](int l, int kmax, hipStream_t s) {
        Lat &L = B.lats[l];
        k_bat_backsub<<<1, 64, 0, s>>>(L.nrhs, L.cyc(), L.cnt(), L.scal(), kmax);
        HIP_CHECK(hipGetLastError());
        // each system sums its own cycle's basis vectors (with a shorter cycle than the batch's,
        // the later slots hold vectors of earlier cycles or calls)
        blas(l).axpy_multi(pr[l], pr[l], 1, x[l], L.w->P.p, kmax, L.sp(S_C), 1.0, s, L.spec(L.cyc()), nullptr,
                           L.cnt() + 2 * L.nrhs);
        // true residuals of the systems that took part in the cycle
        schur_apply(L.c, L.w->Q.p, x[l], 0, pr[l], s, L.nrhs, L.cyc());
        blas(l).lincomb(pr[l], pr[l], pr[l], 1, L.w->r.p, nullptr, 1.0, b[l], -1.0, L.w->Q.p, L.sp(S_RED + 4),
                        scale(l), s, L.spec(L.cyc()));
        k_bat_status<<<1, 64, 0, s>>>(L.nrhs, 2, 0, L.act(), L.cyc(), L.cnt(), L.scal());
        HIP_CHECK(hipGetLastError());
    };
    int it = 0;
    while (active > 0 && it < max_iter) {
        B.run_graph(use_graph, lw.start_graph, [&](bool cap) {
            B.branches(cap, [&](int l, hipStream_t s) { cycle_start(l, s); });
        });
        int kmax = 0;
        for (int k = 0; k < m; ++k) {
            B.run_graph(use_graph, lw.it_graphs[k], [&](bool cap) {
                B.branches(cap, [&](int l, hipStream_t s) { iteration(l, k, s); });
                B.gather(ms);
            });
            ++it;
            kmax = k + 1;
            if (it >= max_iter) break;
            if ((k + 1) % kPoll == 0 && B.poll() == 0) break;
        }
        B.run_graph(use_graph, lw.end_graphs[kmax], [&](bool cap) {
            B.branches(cap, [&](int l, hipStream_t s) { cycle_end(l, kmax, s); });
            B.gather(ms);
        });
        active = B.poll();
    }
    // per-system counters of every lattice
    std::vector<BOut> out(nl);
    std::vector<std::vector<int>> hc(nl);
    for (int l = 0; l < nl; ++l)
        HIP_CHECK(hipMemcpyAsync(pin_ints(B.lats[l]), B.lats[l].cnt(), (4 * B.lats[l].nrhs + 1) * sizeof(int),
                                 hipMemcpyDeviceToHost, ms));
    HIP_CHECK(hipStreamSynchronize(ms));
    ++B.syncs;
    for (int l = 0; l < nl; ++l) hc[l].assign(pin_ints(B.lats[l]), pin_ints(B.lats[l]) + 4 * B.lats[l].nrhs + 1);
    for (int l = 0; l < nl; ++l) {
        const int R = B.lats[l].nrhs;
        BOut &o = out[l];
        o.iters.assign(hc[l].begin(), hc[l].begin() + R);
        o.restarts.assign(hc[l].begin() + R, hc[l].begin() + 2 * R);
        o.converged.resize(R);
        for (int q = 0; q < R; ++q) {
            o.converged[q] = (hc[l][3 * R + q] & 1) != 0;
            if (hc[l][3 * R + q] & 2) o.nonfinite = true;
        }
    }
    B.batch_to_lattices();
    return out;
}

void ensure_bwork(dirac_ctx *c, int m, int nrhs) {
    ensure_work(c, 1, DIRAC_F64, 1);
    c->work->blas.reserve(c->V, kMaxM, nrhs);
    if (!c->bwork) c->bwork = new BWork();
    BWork &w = *c->bwork;
    if (!w.s) HIP_CHECK(hipStreamCreateWithFlags(&w.s, hipStreamNonBlocking));
    const size_t hb = (size_t)nrhs * 24 * 8 * c->g.vhp;  // FP64 (the largest) sizing: fallback needs it
    w.P.alloc(hb * (m + 1));
    w.Q.alloc(hb * m);
    w.r.alloc(hb);
    w.e.alloc(hb);
    w.b.alloc(hb);
    w.act.alloc(nrhs * sizeof(int));
    w.cyc.alloc(nrhs * sizeof(int));
    w.cnt.alloc((4 * nrhs + 1) * sizeof(int));
    w.stage.alloc(kPinDoubles * sizeof(double));
    if (!w.pin) HIP_CHECK(hipHostMalloc((void **)&w.pin, kPinBytes, hipHostMallocDefault));
    for (auto &d : w.h64) d.alloc(hb);
    for (auto &d : w.f64) d.alloc(2 * hb);
}

// The batch-level state of the leading lattice's work space for nlat lattices.
void ensure_lead(BWork &w, const std::vector<Lat> &lats) {
    const int nl = (int)lats.size();
    if (!w.ms) HIP_CHECK(hipStreamCreateWithFlags(&w.ms, hipStreamNonBlocking));
    if (!w.fork) HIP_CHECK(hipEventCreateWithFlags(&w.fork, hipEventDisableTiming));
    while ((int)w.ev.size() < nl) {
        hipEvent_t e;
        HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        w.ev.push_back(e);
    }
    if (w.nlat_cap < nl) {
        if (w.host_nact) HIP_CHECK(hipHostFree(w.host_nact));
        w.host_nact = nullptr;
        HIP_CHECK(hipHostMalloc((void **)&w.host_nact, 64 * sizeof(int), hipHostMallocDefault));
        w.nlat_cap = 64;
    }
    w.table.alloc(64 * sizeof(int *));
    w.nact.alloc(64 * sizeof(int));
    const int **src = (const int **)w.pin;  // the leader's pinned staging (64 pointers fit)
    for (int l = 0; l < nl; ++l) src[l] = (const int *)lats[l].w->cnt.p + 4 * lats[l].nrhs;
    HIP_CHECK(hipMemcpyAsync(w.table.p, src, nl * sizeof(int *), hipMemcpyHostToDevice, w.ms));
    HIP_CHECK(hipStreamSynchronize(w.ms));  // the staging is reused
}

// All lattices: solve D x_r = b_r for nrhs NATIVE FP64 full vectors each (in w.f64[0] -> w.f64[1]).
void solve_all(Batch &B, const dirac_solver_params *p, std::vector<dirac_solve_info *> &info) {
    const int nl = (int)B.lats.size();
    const bool graph = graphs_enabled();
    auto half64 = [&](int l) { return (size_t)24 * 8 * B.lats[l].c->g.vhp; };
    auto scale = [&](int l) { return 1.0 / (24.0 * (double)B.lats[l].c->vh); };
    // split the full vectors into even / odd halves (per system) and back through the half buffers
    auto halves = [&](int l, char *full, void *even, void *odd, bool to_halves) {
        Lat &L = B.lats[l];
        const size_t h = half64(l);
        for (int q = 0; q < L.nrhs; ++q) {
            char *f = full + q * 2 * h;
            hipStream_t s = L.w->s;
            if (to_halves) {
                if (even) HIP_CHECK(hipMemcpyAsync((char *)even + q * h, f, h, hipMemcpyDeviceToDevice, s));
                if (odd) HIP_CHECK(hipMemcpyAsync((char *)odd + q * h, f + h, h, hipMemcpyDeviceToDevice, s));
            } else {
                if (even) HIP_CHECK(hipMemcpyAsync(f, (char *)even + q * h, h, hipMemcpyDeviceToDevice, s));
                if (odd) HIP_CHECK(hipMemcpyAsync(f + h, (char *)odd + q * h, h, hipMemcpyDeviceToDevice, s));
            }
        }
    };
    std::vector<std::vector<double>> target(nl), bn(nl);
    std::vector<std::vector<int>> live(nl), all(nl);
    for (int l = 0; l < nl; ++l) {
        Lat &L = B.lats[l];
        dirac_ctx *c = L.c;
        hipStream_t s = L.w->s;
        Blas &Bl = c->work->blas;
        const int R = L.nrhs;
        require(c->f[DIRAC_F64].inv_ready[1], "odd-site clover inverse not available");
        all[l].assign(R, 1);
        upload_mask(L, all[l], L.act(), s);
        // |b_r|
        Bl.mdot(DIRAC_F64, 2, L.w->f64[0].p, 1, L.w->f64[0].p, L.sp(S_MISC), scale(l), s, L.spec(L.act()));
        // eta-hat_e = b_e - D_eo A_oo^-1 b_o (all systems): even halves into eta, odd into r64
        void *eta = L.w->h64[0].p, *r64 = L.w->h64[2].p, *t64 = L.w->h64[3].p;
        halves(l, (char *)L.w->f64[0].p, eta, r64, true);
        clover_apply(c, t64, r64, 1, 1, DIRAC_F64, s, R);
        hop_apply(c, r64, t64, nullptr, 0, HOP_PLAIN, -0.5, 0, DIRAC_F64, s, R);
        Bl.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, eta, nullptr, 1.0, eta, -1.0, r64, nullptr, 1.0, s,
                   L.spec(L.act()));
    }
    for (int l = 0; l < nl; ++l) {
        Lat &L = B.lats[l];
        read_sys(L, S_MISC, bn[l], L.w->s);
        ++B.syncs;
        target[l].resize(L.nrhs);
        live[l].resize(L.nrhs);
        for (int q = 0; q < L.nrhs; ++q) {
            bn[l][q] = std::sqrt(bn[l][q]);
            require(std::isfinite(bn[l][q]), "right-hand side holds NaN or Inf", DIRAC_ENONFINITE);
            target[l][q] = p->tol * bn[l][q];
            live[l][q] = bn[l][q] > 0.0;
        }
    }
    std::vector<void *> xe(nl), ee(nl);
    std::vector<const void *> eta(nl), bb(nl);
    for (int l = 0; l < nl; ++l) {
        xe[l] = B.lats[l].w->h64[1].p;
        eta[l] = B.lats[l].w->h64[0].p;
        ee[l] = B.lats[l].w->e.p;
        bb[l] = B.lats[l].w->b.p;
    }
    if (p->method == DIRAC_SOLVER_GCR) {
        std::vector<BOut> o = gcr_batched(B, std::vector<dirac_prec>(nl, DIRAC_F64), xe, eta, live, target, p->restart,
                                          p->max_iter, graph);
        for (int l = 0; l < nl; ++l)
            for (int q = 0; q < B.lats[l].nrhs; ++q) {
                info[l][q].iters = o[l].iters[q];
                info[l][q].restarts = o[l].restarts[q];
            }
    } else {
        // defect correction per system around the batched inner GCR, all lattices in step
        std::vector<dirac_prec> cur(nl, (dirac_prec)p->inner_prec);
        const dirac_prec p0 = (dirac_prec)p->inner_prec;
        const double dtol = p->inner_tol > 0.0 ? p->inner_tol : (p0 == DIRAC_F32 ? 1e-5 : p0 == DIRAC_F16 ? 1e-3 : 1e-2);
        std::vector<std::vector<double>> rn(nl), itarget(nl);
        std::vector<std::vector<int>> outer(nl);
        for (int l = 0; l < nl; ++l) {
            Lat &L = B.lats[l];
            hipStream_t s = L.w->s;
            Blas &Bl = L.c->work->blas;
            ensure_prec(L.c, cur[l], s);
            Bl.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, xe[l], nullptr, 0.0, eta[l], 0.0, nullptr, nullptr, 1.0, s,
                       L.spec(L.act()));
            Bl.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, L.w->h64[2].p, nullptr, 1.0, eta[l], 0.0, nullptr,
                       L.sp(S_MISC + 2), scale(l), s, L.spec(L.act()));
            read_sys(L, S_MISC + 2, rn[l], s);
            ++B.syncs;
            for (auto &v : rn[l]) v = std::sqrt(v);
            itarget[l].assign(L.nrhs, dtol);
            outer[l].resize(L.nrhs);
        }
        int used = 0;
        while (true) {
            bool anyo = false;
            for (int l = 0; l < nl; ++l)
                for (int q = 0; q < B.lats[l].nrhs; ++q) {
                    outer[l][q] = live[l][q] && rn[l][q] > target[l][q] && std::isfinite(rn[l][q]);
                    anyo = anyo || outer[l][q];
                }
            if (!anyo || used >= p->max_iter) break;
            // lattices whose inner precision went up to FP64 finish with plain FP64 GCR on the
            // correction D-hat e = r from their current iterates; the others take one more
            // defect-correction step in their inner precision
            std::vector<std::vector<int>> start(nl);
            std::vector<std::vector<double>> tg(nl);
            std::vector<const void *> rhs(nl);
            for (int l = 0; l < nl; ++l) {
                Lat &L = B.lats[l];
                hipStream_t s = L.w->s;
                start[l] = outer[l];
                if (cur[l] == DIRAC_F64) {
                    tg[l] = target[l];
                    rhs[l] = L.w->h64[2].p;  // r64
                } else {
                    std::vector<double> inv(L.nrhs);
                    for (int q = 0; q < L.nrhs; ++q) inv[q] = outer[l][q] ? 1.0 / rn[l][q] : 0.0;
                    write_sys(L, S_ALPHA, inv, s);
                    upload_mask(L, outer[l], L.act(), s);
                    L.c->work->blas.lincomb(cur[l], DIRAC_F64, DIRAC_F64, 1, L.w->b.p, nullptr, 1.0, L.w->h64[2].p,
                                            0.0, nullptr, nullptr, 1.0, s, L.spec(L.act()), L.sp(S_ALPHA));
                    tg[l] = itarget[l];
                    rhs[l] = bb[l];
                }
            }
            std::vector<BOut> o = gcr_batched(B, cur, ee, rhs, start, tg, p->restart, p->max_iter - used, graph);
            int mx = 0;
            for (int l = 0; l < nl; ++l)
                for (int q = 0; q < B.lats[l].nrhs; ++q) {
                    info[l][q].iters += o[l].iters[q];
                    info[l][q].restarts += o[l].restarts[q];
                    if (outer[l][q]) {
                        if (cur[l] == DIRAC_F64) info[l][q].fell_back = 1;
                        else ++info[l][q].outer;
                    }
                    mx = std::max(mx, o[l].iters[q]);
                }
            used += mx;
            bool done = true;
            for (int l = 0; l < nl; ++l) {
                Lat &L = B.lats[l];
                hipStream_t s = L.w->s;
                Blas &Bl = L.c->work->blas;
                const int R = L.nrhs;
                // x_e += e (FP64 correction) or x_e += rn_r e_r (scaled inner solution)
                write_sys(L, S_XS, cur[l] == DIRAC_F64 ? std::vector<double>(R, 1.0) : rn[l], s);
                write_sys(L, S_ONE, std::vector<double>(R, 1.0), s);
                write_sys(L, S_ONE + 1, std::vector<double>(R, 0.0), s);
                upload_mask(L, outer[l], L.act(), s);
                Bl.axpy_multi(DIRAC_F64, cur[l], 1, xe[l], ee[l], 1, L.sp(S_ONE), 1.0, s, L.spec(L.act()), L.sp(S_XS));
                if (cur[l] == DIRAC_F64) continue;  // finished: nothing more for this lattice
                done = false;
                void *t64 = L.w->h64[3].p;
                schur_apply(L.c, t64, xe[l], 0, DIRAC_F64, s, R, L.act());
                Bl.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, L.w->h64[2].p, nullptr, 1.0, eta[l], -1.0, t64,
                           L.sp(S_MISC + 2), scale(l), s, L.spec(L.act()));
            }
            for (int l = 0; l < nl; ++l) {
                Lat &L = B.lats[l];
                if (cur[l] == DIRAC_F64) {
                    // the FP64 solve ended this lattice's systems
                    for (int q = 0; q < L.nrhs; ++q) outer[l][q] = 0;
                    for (int q = 0; q < L.nrhs; ++q) live[l][q] = 0;
                    continue;
                }
                std::vector<double> rnew;
                read_sys(L, S_MISC + 2, rnew, L.w->s);
                ++B.syncs;
                bool stalled = o[l].nonfinite;
                for (int q = 0; q < L.nrhs; ++q) {
                    if (!outer[l][q]) continue;
                    rnew[q] = std::sqrt(rnew[q]);
                    if (!(rnew[q] < 0.5 * rn[l][q])) stalled = true;
                    rn[l][q] = rnew[q];
                }
                if (stalled) cur[l] = cur[l] == DIRAC_F32 ? DIRAC_F64 : DIRAC_F32;  // raise the inner precision
                if (cur[l] != DIRAC_F64) ensure_prec(L.c, cur[l], L.w->s);
            }
            if (done) break;
        }
    }
    // x_o = A_oo^-1 (b_o - D_oe x_e); assemble the full solutions; a-posteriori residuals
    for (int l = 0; l < nl; ++l) {
        Lat &L = B.lats[l];
        dirac_ctx *c = L.c;
        hipStream_t s = L.w->s;
        Blas &Bl = c->work->blas;
        const int R = L.nrhs;
        void *r64 = L.w->h64[2].p, *t64 = L.w->h64[3].p;
        char *bf = (char *)L.w->f64[0].p, *xf = (char *)L.w->f64[1].p, *rf = (char *)L.w->f64[2].p;
        const size_t full64 = 2 * half64(l);
        halves(l, bf, nullptr, r64, true);  // r64 <- b_o
        hop_apply(c, t64, xe[l], nullptr, 1, HOP_PLAIN, -0.5, 0, DIRAC_F64, s, R);
        upload_mask(L, all[l], L.act(), s);
        Bl.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 1, r64, nullptr, 1.0, r64, -1.0, t64, nullptr, 1.0, s,
                   L.spec(L.act()));
        clover_apply(c, t64, r64, 1, 1, DIRAC_F64, s, R);
        halves(l, xf, xe[l], t64, false);
        for (int q = 0; q < R; ++q) full_apply(c, rf + q * full64, xf + q * full64, 0, DIRAC_F64, s);
        Bl.lincomb(DIRAC_F64, DIRAC_F64, DIRAC_F64, 2, rf, nullptr, 1.0, bf, -1.0, rf, L.sp(S_MISC + 4), scale(l), s,
                   L.spec(L.act()));
    }
    for (int l = 0; l < nl; ++l) {
        Lat &L = B.lats[l];
        std::vector<double> tr;
        read_sys(L, S_MISC + 4, tr, L.w->s);
        ++B.syncs;
        for (int q = 0; q < L.nrhs; ++q)
            info[l][q].true_rel_res = bn[l][q] > 0.0 ? std::sqrt(tr[q]) / bn[l][q] : 0.0;
    }
}

}  // namespace

void free_bwork(dirac_ctx *c) {
    if (c->bwork) {
        delete c->bwork;
        c->bwork = nullptr;
    }
}

// Solve all lattices from this thread.  x[l] / b[l] hold nrhs consecutive full-lattice FP64 vectors
// in `lay`.  Work is queued behind what the caller already put on its stream.
dirac_status solve_batched(dirac_ctx *const *ctx, int nlat, void *const *x, const void *const *b, int nrhs,
                           dirac_layout lay, const dirac_solver_params *p, dirac_solve_info *info, hipStream_t user,
                           std::string &err) {
    const auto t0 = std::chrono::steady_clock::now();
    Batch B;
    for (int l = 0; l < nlat; ++l) {
        ensure_bwork(ctx[l], p->restart, nrhs);
        B.lats.push_back(Lat{ctx[l], ctx[l]->bwork, nrhs});
    }
    B.lead = ctx[0]->bwork;
    if (const char *e = getenv("DIRAC_BATCH_CONCURRENT")) B.concurrent = atoi(e) != 0;
    ensure_lead(*B.lead, B.lats);
    hipEvent_t ready;
    HIP_CHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIP_CHECK(hipEventRecord(ready, user));
    std::vector<dirac_solve_info *> inf(nlat);
    for (int l = 0; l < nlat; ++l) {
        dirac_ctx *c = ctx[l];
        BWork &w = *c->bwork;
        HIP_CHECK(hipStreamWaitEvent(w.s, ready, 0));
        const size_t full64 = (size_t)48 * 8 * c->g.vhp;
        const size_t ub = (size_t)c->V * 24 * 8;
        for (int q = 0; q < nrhs; ++q) {
            char *dst = (char *)w.f64[0].p + q * full64;
            if (lay == DIRAC_LAYOUT_NATIVE)
                HIP_CHECK(hipMemcpyAsync(dst, (const char *)b[l] + q * full64, full64, hipMemcpyDeviceToDevice, w.s));
            else
                spinor_import(c, dst, (const char *)b[l] + q * ub, 0, DIRAC_F64, lay, w.s);
        }
        inf[l] = info + (size_t)l * nrhs;
        for (int q = 0; q < nrhs; ++q) inf[l][q] = dirac_solve_info{};
    }
    try {
        solve_all(B, p, inf);
    } catch (...) {
        // leave no work of this call queued behind the caller's back
        for (auto &L : B.lats) (void)hipStreamSynchronize(L.w->s);
        (void)hipStreamSynchronize(B.ms());
        (void)hipEventDestroy(ready);
        throw;
    }
    for (int l = 0; l < nlat; ++l) {
        dirac_ctx *c = ctx[l];
        BWork &w = *c->bwork;
        const size_t full64 = (size_t)48 * 8 * c->g.vhp;
        const size_t ub = (size_t)c->V * 24 * 8;
        for (int q = 0; q < nrhs; ++q) {
            char *src = (char *)w.f64[1].p + q * full64;
            if (lay == DIRAC_LAYOUT_NATIVE)
                HIP_CHECK(hipMemcpyAsync((char *)x[l] + q * full64, src, full64, hipMemcpyDeviceToDevice, w.s));
            else
                spinor_export(c, (char *)x[l] + q * ub, src, 0, DIRAC_F64, lay, w.s);
        }
    }
    for (auto &L : B.lats) HIP_CHECK(hipStreamSynchronize(L.w->s));
    ++B.syncs;
    // destroyed only now: the lattice streams' waits on it have run (a wait on an event destroyed
    // before the wait executes need not order anything)
    (void)hipEventDestroy(ready);
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    dirac_status st = DIRAC_OK;
    for (int l = 0; l < nlat; ++l)
        for (int q = 0; q < nrhs; ++q) {
            inf[l][q].seconds = sec;
            inf[l][q].host_syncs = (int)B.syncs;
            if (!std::isfinite(inf[l][q].true_rel_res)) {
                if (st == DIRAC_OK) err = "lattice " + std::to_string(l) + ": a system met NaN or Inf";
                st = DIRAC_ENONFINITE;
            } else if (!(inf[l][q].true_rel_res < p->tol) && st == DIRAC_OK) {
                st = DIRAC_ENOCONV;
                err = "lattice " + std::to_string(l) + ": a system did not reach the tolerance";
            }
        }
    return st;
}

}  // namespace dl
