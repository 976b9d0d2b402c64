// Host runtime behind the C ABI of include/qap_swarm.h: parameter checks,
// range checks and path choice, device buffers, the per-iteration launch
// sequence (or its HIP graph), state import/export.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdio>
#include <mutex>
#include <string>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "qap_swarm.h"

using qap::InstDesc;

namespace {

// Swarms on the fused kernel are stepped as concurrent chains of launches,
// each on its own stream (the device has 4 hardware queues per process): one
// chain's end-of-iteration tail overlaps another chain's work.  The default is
// 3 chains, each holding a slice of every instance's swarms (measured: 3
// chains step the 10,000-particle n = 128 workload about 20 % faster than one).
constexpr int kStreamGroups = 3;
constexpr int kMaxChains = QAP_MAX_CHAINS;

// Iterations captured into one graph: consecutive launches of one graph run
// back to back on the device, while each new graph launch on a stream starts
// about 0.1 ms after the previous one ended (measured on the 64-instance
// batch), so steps replay graphs of several iterations.
constexpr int kItersPerGraph = 8;

struct Instance {
    InstDesc d{};                 // the whole instance (iteration 0, state import/export, eval)
    int n = 0, m = 0, S = 0, P = 0;
    int mul24 = 0;
    bool stepped = false;         // a step ran since init / set_state: the buffers of the previous state hold it
    long long t = 0;              // completed iterations (host copy of the device counter)
    // per-iteration statistics (qap_swarm_history_start): ring of records
    int hist_cap = 0, hist_nq = 0, hist_bins = 0;
    long long hist_lo = 0, hist_hi = 1, hist_t0 = 0;  // hist_t0: iteration when recording started
    long long* hist_ranks = nullptr;       // device [(m + 1) nq]
    int* ring_t = nullptr;                 // device [cap]
    long long* ring_q = nullptr;           // device [cap][m + 1][nq]
    unsigned long long* ring_h = nullptr;  // device [cap][m + 1][bins]
    int* order = nullptr;         // [m] migration ranking scratch
    int groups = 1;               // swarm groups of the instance under the current plan
    std::vector<InstDesc> gdesc;  // [groups] descriptor of each group's swarms
    std::vector<int> chain;       // [groups] launch chain (stream) of each group
    int param_groups = 0;         // stream_groups of the instance's parameters (0: automatic)
    std::vector<void*> allocs;
};

// Device tables of one step over all instances of a handle: every descriptor,
// the swarm map of the batched bests, and per fused-kernel class (npad,
// symmetric, zero diagonals) its descriptors and workgroup map.
struct FusedClass {
    int npad = 0;
    int wide = 0;  // 0 int8, else the byte-split pattern (1 F split, 2 D split, 3 both)
    bool sym = false, zd = false;
    int blocks = 0;
    qap::InstDesc* descs = nullptr;  // device [instances of the class]
    int2* blkmap = nullptr;          // device [blocks]: (class-local instance, first particle)
    std::vector<qap::InstDesc> host; // the class's descriptors (one instance: passed by value)
};

struct StepPlan {
    qap::InstDesc* descs = nullptr;  // device [instances]
    int2* smap = nullptr;            // device [total swarms]: (descriptor, swarm)
    int total_swarms = 0;
    int count = 0;                   // descriptors
    std::vector<FusedClass> fused;
    std::vector<int> plain;          // instances stepped by the per-stage kernels
    std::vector<void*> allocs;
};

}  // namespace

// A launch plan: how the iterations of a handle are spread over streams and
// launched.  Results do not depend on it (states are bit-identical).
struct PlanCfg {
    int chains = kStreamGroups;  // concurrent launch chains, 1..kMaxChains
    int split = 0;               // 0: every instance's swarms over the chains; 1: whole instances; 2: whole classes
    int ipg = 8;                 // iterations per captured graph; 0: eager launches
};

struct qap_swarm {
    std::vector<Instance> inst;
    PlanCfg cfg;
    StepPlan init;                        // whole instances: iteration 0
    std::vector<StepPlan> plans;          // one per stream group
    std::vector<hipStream_t> gstream;     // [groups]; gstream[0] = stream, the others owned
    std::vector<hipEvent_t> gevent;       // [groups]: fork (0) and joins (1..)
    std::vector<hipGraphExec_t> graphs;   // [groups] one iteration each, captured at the first step
    std::vector<hipGraphExec_t> graphs_k; // [groups] cfg.ipg iterations each
    std::vector<int> migr;                // instances in migration mode stepped in several groups
    qap::InstDesc* migr_descs = nullptr;  // device [migr.size()]: their whole-instance descriptors
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* scratch = nullptr;              // device address of the stats scratch array on this device
    int engine = QAP_ENGINE_PLAIN;
    int sticky = QAP_OK;
    int grid_gd = 0;
    int device = 0;
    bool graph_failed = false;            // capture unavailable on a stream: eager launches
    // profiled stepping
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;   // sets of 2 * QAP_NUM_STAGES events
    std::vector<uint8_t> ev_mask;      // per set: stages recorded since the set was handed out
    size_t ev_used = 0;
    double stage_ms[QAP_NUM_STAGES] = {};
    long long prof_iters = 0;
};

namespace {

// Every device allocation of the library goes through dev_malloc / dev_free:
// a count of the blocks held (qap_swarm_live_allocations) and the
// allocation-failure injection of qap_swarm_fail_alloc.
std::atomic<long long> g_live_allocs{0};
std::atomic<long long> g_fail_countdown{0};

hipError_t dev_malloc(void** p, size_t bytes)
{
    *p = nullptr;
    long long c = g_fail_countdown.load();
    while (c > 0 && !g_fail_countdown.compare_exchange_weak(c, c - 1)) {
    }
    if (c == 1) return hipErrorOutOfMemory;  // the injected failure
    const hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 1);
    if (e == hipSuccess) g_live_allocs.fetch_add(1);
    else *p = nullptr;
    return e;
}

void dev_free(void* p)
{
    if (!p) return;
    (void)hipFree(p);
    g_live_allocs.fetch_sub(1);
}

// Scratch of qap_swarm_stats_noalloc: a fixed device array (each GPU holds
// its own copy until the process ends).  In host code the name `scratch` is a
// host-side stand-in; the device address is taken once per device, with that
// device current, by hipGetSymbolAddress at the first init on the device, and
// only that address is used from then on.
constexpr size_t kScratchBytes = QAP_STATS_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
hipError_t scratch_address(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// A failed allocation leaves the handle usable (nothing ran); any other
// device error is sticky.
int dev_err(qap_swarm* h, hipError_t e)
{
    if (e == hipSuccess) return QAP_OK;
    if (e == hipErrorOutOfMemory) return QAP_ERR_NOMEM;
    if (h) h->sticky = QAP_ERR_DEVICE;
    return QAP_ERR_DEVICE;
}

template <class T>
hipError_t dalloc(Instance& I, T** p, size_t count)
{
    void* q = nullptr;
    hipError_t e = dev_malloc(&q, count * sizeof(T));
    if (e != hipSuccess) { *p = nullptr; return e; }
    I.allocs.push_back(q);
    *p = static_cast<T*>(q);
    return hipSuccess;
}

void free_history(Instance& I)
{
    dev_free(I.hist_ranks);
    dev_free(I.ring_t);
    dev_free(I.ring_q);
    dev_free(I.ring_h);
    I.hist_ranks = nullptr;
    I.ring_t = nullptr;
    I.ring_q = nullptr;
    I.ring_h = nullptr;
    I.hist_cap = 0;
}

void free_instance(Instance& I)
{
    free_history(I);
    for (void* p : I.allocs) dev_free(p);
    I.allocs.clear();
}

int check_params(const qap_instance* in, const qap_params* p)
{
    if (!in || !p || !in->F || !in->D) return QAP_ERR_INVALID_ARG;
    const int n = in->n;
    if (n < 2 || n > qap::kMaxN) return QAP_ERR_INVALID_ARG;
    if (p->num_swarms < 1 || p->particles_per_swarm < 1) return QAP_ERR_INVALID_ARG;
    if ((long long)p->num_swarms * p->particles_per_swarm > (1LL << 24)) return QAP_ERR_INVALID_ARG;
    const float cs[3] = {p->c1, p->c2, p->c3};
    for (float c : cs)
        if (!(c >= 0.0f && c <= 1.0f)) return QAP_ERR_INVALID_ARG;
    if (!(p->vmax > 0.0f) || !(p->vmax < 1e30f)) return QAP_ERR_INVALID_ARG;
    if (p->velocity_kernel != QAP_SV_RAW && p->velocity_kernel != QAP_SV_NORM) return QAP_ERR_INVALID_ARG;
    if (p->st_depth < 0 || p->st_depth > n - 1) return QAP_ERR_INVALID_ARG;
    if (p->mode != QAP_INDEPENDENT && p->mode != QAP_MIGRATION) return QAP_ERR_INVALID_ARG;
    if (p->mode == QAP_MIGRATION) {
        if (!(p->migration_factor >= 0.0f) || p->migration_period < 1) return QAP_ERR_INVALID_ARG;
        const long long d = (long long)(p->migration_factor * (float)p->num_swarms);
        if (2 * d >= p->num_swarms && d > 0) return QAP_ERR_INVALID_ARG;
    }
    if (p->local_search < 0 || p->local_search > QAP_MAX_EXCHANGES) return QAP_ERR_INVALID_ARG;
    if (p->delta_path < QAP_PATH_AUTO || p->delta_path > QAP_PATH_SPLIT_MFMA) return QAP_ERR_INVALID_ARG;
    if (p->engine != QAP_ENGINE_FUSED && p->engine != QAP_ENGINE_PLAIN) return QAP_ERR_INVALID_ARG;
    if (p->stream_groups < 0 || p->stream_groups > kMaxChains) return QAP_ERR_INVALID_ARG;
    if (p->sx_procedure != QAP_SX_SECOND_TARGET && p->sx_procedure != QAP_SX_PICK_COLUMN) return QAP_ERR_INVALID_ARG;
    return QAP_OK;
}

// Range check and path choice.  int8 MFMA needs every entry in [-128, 127];
// any exact int32 contraction needs n * max|F| * max|D| < 2^31.  The
// byte-split MFMA path needs F and D symmetric, every entry in
// [-16384, 16383] (two planes of 7 + 8 bits) and 8 (n + 3) max|F| max|D| <
// 2^31, which bounds every delta (at most 8 (n + 2) max|F| max|D| in size) and
// every partial sum of its int32 epilogue.
int choose_path(const qap_instance* in, const qap_params* p, int engine, int* path, int* sym, int* mul24,
                int* zd, int* split)
{
    const int n = in->n;
    long long mf = 0, md = 0;
    bool f8 = true, s = true, z = true, fs = false, ds = false, w15 = true;
    for (int i = 0; i < n; ++i) z = z && in->F[i * n + i] == 0 && in->D[i * n + i] == 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const long long f = in->F[i * n + j], dd = in->D[i * n + j];
            mf = std::max(mf, f < 0 ? -f : f);
            md = std::max(md, dd < 0 ? -dd : dd);
            if (f < -128 || f > 127 || dd < -128 || dd > 127) f8 = false;
            fs = fs || f < -128 || f > 127;
            ds = ds || dd < -128 || dd > 127;
            w15 = w15 && f >= -16384 && f <= 16383 && dd >= -16384 && dd <= 16383;
            if (in->F[i * n + j] != in->F[j * n + i] || in->D[i * n + j] != in->D[j * n + i]) s = false;
        }
    if ((long long)n * mf * md >= (1LL << 31)) return QAP_ERR_RANGE;
    const bool fused = engine == QAP_ENGINE_FUSED && n <= 160 && p->sx_procedure == QAP_SX_SECOND_TARGET;
    // split pattern: bit 0 F, bit 1 D; the byte-split path asked for on data
    // that fits int8 splits F (exactly: its high plane holds 0 or -1)
    const int spl = (fs || !ds ? 1 : 0) | (ds ? 2 : 0);
    const bool split_ok = s && w15 && 8LL * (n + 3) * mf * md < (1LL << 31) &&
                          qap::split_supported((n + 31) / 32 * 32, spl);
    int pth;
    if (p->delta_path == QAP_PATH_INT8_MFMA) {
        if (!f8) return QAP_ERR_RANGE;
        pth = 1;
    } else if (p->delta_path == QAP_PATH_SPLIT_MFMA) {
        if (!split_ok) return QAP_ERR_RANGE;
        pth = 3;
    } else if (p->delta_path == QAP_PATH_INT32) {
        pth = 2;
    } else {
        pth = f8 ? 1 : split_ok && fused ? 3 : 2;
    }
    if (!fused) pth = 2;  // the fused kernels cover SecondTarget with n <= 160
    *path = pth;
    *sym = s ? 1 : 0;
    *mul24 = (mf < (1LL << 23) && md < (1LL << 23)) ? 1 : 0;
    *zd = z ? 1 : 0;
    *split = pth == 3 ? spl : 0;
    return QAP_OK;
}

int init_state(qap_swarm* h, Instance& I);

int setup_instance(qap_swarm* h, Instance& I, const qap_instance* in, const qap_params* p, int path, int sym,
                   int mul24, int zd, int split)
{
    const int n = in->n;
    InstDesc& d = I.d;
    I.n = n;
    I.m = p->num_swarms;
    I.S = p->particles_per_swarm;
    I.P = I.m * I.S;
    I.mul24 = mul24;
    d.n = n;
    d.npad = (n + 31) / 32 * 32;
    d.m = I.m;
    d.S = I.S;
    d.P = I.P;
    d.c1 = p->c1; d.c2 = p->c2; d.c3 = p->c3; d.vmax = p->vmax;
    d.norm = p->velocity_kernel == QAP_SV_NORM;
    d.depth = p->st_depth;
    d.sx = p->sx_procedure;
    d.ls = p->local_search;
    d.migrate = p->mode == QAP_MIGRATION;
    d.migr_d = d.migrate ? (int)(p->migration_factor * (float)I.m) : 0;
    d.period = p->migration_period < 1 ? 1 : p->migration_period;
    d.sym = sym;
    d.zd = zd;
    d.path = path;
    d.split = split;
    d.seed = p->seed;
    const size_t nn = (size_t)n * n, P = (size_t)I.P;
    hipError_t e = hipSuccess;
    int* F32 = nullptr; int* D32 = nullptr;
#define TRY(x) do { e = (x); if (e != hipSuccess) return dev_err(nullptr, e); } while (0)
    TRY(dalloc(I, &F32, nn));
    TRY(dalloc(I, &D32, nn));
    TRY(hipMemcpy(F32, in->F, nn * sizeof(int), hipMemcpyHostToDevice));
    TRY(hipMemcpy(D32, in->D, nn * sizeof(int), hipMemcpyHostToDevice));
    d.F32 = F32; d.D32 = D32;
    if (path == 1) {
        const size_t np = (size_t)d.npad;
        std::vector<int8_t> hF(np * np, 0), hD(np * np, 0), hFT(np * np, 0), hDT(np * np, 0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                hF[i * np + j] = (int8_t)in->F[i * n + j];
                hD[i * np + j] = (int8_t)in->D[i * n + j];
                hFT[j * np + i] = (int8_t)in->F[i * n + j];
                hDT[j * np + i] = (int8_t)in->D[i * n + j];
            }
        int8_t *F8, *D8, *FT8, *DT8;
        TRY(dalloc(I, &F8, np * np));
        TRY(dalloc(I, &D8, np * np));
        TRY(dalloc(I, &FT8, np * np));
        TRY(dalloc(I, &DT8, np * np));
        TRY(hipMemcpy(F8, hF.data(), np * np, hipMemcpyHostToDevice));
        TRY(hipMemcpy(D8, hD.data(), np * np, hipMemcpyHostToDevice));
        TRY(hipMemcpy(FT8, hFT.data(), np * np, hipMemcpyHostToDevice));
        TRY(hipMemcpy(DT8, hDT.data(), np * np, hipMemcpyHostToDevice));
        d.F8 = F8; d.D8 = D8; d.FT8 = FT8; d.DT8 = DT8;
    } else if (path == 3) {
        // planes of F and D (both symmetric): low = M mod 128 and high =
        // floor(M / 128) for a split matrix, low = M otherwise
        const size_t np = (size_t)d.npad;
        const int* src[2] = {in->F, in->D};
        const int8_t** lo[2] = {&d.F8, &d.D8};
        const int8_t** hi[2] = {&d.FH8, &d.DH8};
        for (int m = 0; m < 2; ++m) {
            const bool sp = (split >> m) & 1;
            std::vector<int8_t> hl(np * np, 0), hh(np * np, 0);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    const int v = src[m][i * n + j];
                    const int low = sp ? (v & 127) : v;
                    hl[i * np + j] = (int8_t)low;
                    hh[i * np + j] = (int8_t)((v - low) / 128);
                }
            int8_t *L, *H = nullptr;
            TRY(dalloc(I, &L, np * np));
            TRY(hipMemcpy(L, hl.data(), np * np, hipMemcpyHostToDevice));
            if (sp) {
                TRY(dalloc(I, &H, np * np));
                TRY(hipMemcpy(H, hh.data(), np * np, hipMemcpyHostToDevice));
            }
            *lo[m] = L;
            *hi[m] = H;
        }
    }
    const size_t nv = (size_t)n * n;
    TRY(dalloc(I, &d.V[0], P * nv));
    TRY(dalloc(I, &d.V[1], P * nv));
    TRY(dalloc(I, &d.Vinv[0], P * n));
    TRY(dalloc(I, &d.Vinv[1], P * n));
    TRY(dalloc(I, &d.X[0], P * n));
    TRY(dalloc(I, &d.X[1], P * n));
    TRY(dalloc(I, &d.PL, P * n));
    TRY(dalloc(I, &d.Xnew, P * n));
    TRY(hipMemset(d.Xnew, 0, P * n));
    TRY(dalloc(I, &d.goal, P));
    TRY(dalloc(I, &d.goalPL, P));
    TRY(dalloc(I, &d.PG, (size_t)I.m * n));
    TRY(dalloc(I, &d.goalPG, (size_t)I.m));
    TRY(dalloc(I, &d.smin, (size_t)I.m));
    I.param_groups = p->stream_groups;
    TRY(dalloc(I, &d.best, (size_t)kMaxChains));
    TRY(dalloc(I, &d.iter, (size_t)kMaxChains));
    TRY(dalloc(I, &I.order, (size_t)I.m));
    d.order = I.order;
    TRY(dalloc(I, &d.scratch, (size_t)h->grid_gd * nn * (sym ? 1 : 2)));
#undef TRY
    return init_state(h, I);
}

// Iteration 0 of an instance on the handle's stream (the bests follow, batched
// over the handle): no swarm best yet, empty best-ever records, counters at 0,
// random permutations and velocities, their goals.
int init_state(qap_swarm* h, Instance& I)
{
    const InstDesc& d = I.d;
    std::vector<long long> big((size_t)I.m, LLONG_MAX);
    hipError_t e = hipMemcpy(d.goalPG, big.data(), sizeof(long long) * I.m, hipMemcpyHostToDevice);
    std::vector<qap::BestRec> none((size_t)kMaxChains);
    for (qap::BestRec& r : none) {
        std::memset(&r, 0, sizeof r);
        r.goal = LLONG_MAX;
    }
    if (e == hipSuccess) e = hipMemcpy(d.best, none.data(), sizeof(qap::BestRec) * kMaxChains, hipMemcpyHostToDevice);
    const std::vector<int> zeros((size_t)kMaxChains, 0);
    if (e == hipSuccess) e = hipMemcpy(d.iter, zeros.data(), sizeof(int) * kMaxChains, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = qap::launch_init(d, h->stream);
    if (e == hipSuccess)
        e = qap::launch_goal_delta_i32(d, I.mul24, h->grid_gd, d.X[0], I.P, 2, nullptr, nullptr, h->stream);
    I.t = 0;
    I.stepped = false;
    return dev_err(nullptr, e);
}

// Group descriptors of an instance under a plan: swarms [g0, g0 + mj) of
// group j seen as an instance of their own, with its own iteration counter
// and best-ever record.
void make_groups(Instance& I, int groups)
{
    const InstDesc& d = I.d;
    const size_t n = (size_t)I.n, nv = n * n;
    I.groups = groups;
    I.gdesc.clear();
    for (int j = 0, g0 = 0; j < I.groups; ++j) {
        const int mj = I.m / I.groups + (j < I.m % I.groups ? 1 : 0);
        const size_t p0 = (size_t)g0 * I.S;
        qap::InstDesc gd = d;
        gd.swarm_base = g0;
        gd.m = mj;
        gd.P = mj * I.S;
        for (int b = 0; b < 2; ++b) {
            gd.V[b] = d.V[b] + p0 * nv;
            gd.Vinv[b] = d.Vinv[b] + p0 * n;
            gd.X[b] = d.X[b] + p0 * n;
        }
        gd.PL = d.PL + p0 * n;
        gd.goal = d.goal + p0;
        gd.goalPL = d.goalPL + p0;
        gd.PG = d.PG + (size_t)g0 * n;
        gd.goalPG = d.goalPG + g0;
        gd.smin = d.smin + g0;
        gd.order = d.order + g0;
        gd.Xnew = d.Xnew + p0 * n;
        gd.iter = d.iter + j;
        gd.best = d.best + j;
        // Alg. 2 ranks every swarm of the instance: with several groups it
        // runs once all groups have finished the iteration (qap_swarm_step)
        if (I.groups > 1) {
            gd.migrate = 0;
            gd.migr_d = 0;
        }
        I.gdesc.push_back(gd);
        g0 += mj;
    }
}

template <class T>
hipError_t plan_upload(StepPlan& pl, T** p, const std::vector<T>& v)
{
    void* q = nullptr;
    hipError_t e = dev_malloc(&q, v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    pl.allocs.push_back(q);
    *p = static_cast<T*>(q);
    if (v.empty()) return hipSuccess;
    return hipMemcpy(q, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

void free_plan(StepPlan& pl)
{
    for (void* p : pl.allocs) dev_free(p);
    pl = StepPlan();
}

int fused_kind(const qap::InstDesc& d) { return d.path != 3 ? 0 : d.split; }

// Device tables of one step over the descriptors descs (entry i belongs to
// instance owner[i]); instances whose entry is not on the fused kernel go to
// the per-stage list.
int build_plan(qap_swarm* h, StepPlan& pl, const std::vector<qap::InstDesc>& all, const std::vector<int>& owner)
{
    const int count = (int)all.size();
    pl.count = count;
    std::vector<int2> smap;
    for (int k = 0; k < count; ++k)
        for (int g = 0; g < all[(size_t)k].m; ++g) smap.push_back(make_int2(k, g));
    pl.total_swarms = (int)smap.size();
    hipError_t e = plan_upload(pl, &pl.descs, all);
    if (e == hipSuccess) e = plan_upload(pl, &pl.smap, smap);
    if (e != hipSuccess) return dev_err(nullptr, e);
    // fused classes, larger matrices first
    std::vector<std::vector<int>> members;
    for (int k = 0; k < count; ++k) {
        const qap::InstDesc& d = all[(size_t)k];
        if (h->engine != QAP_ENGINE_FUSED || !qap::fused_supported(d)) {
            pl.plain.push_back(owner[(size_t)k]);
            continue;
        }
        size_t c = 0;
        while (c < pl.fused.size() &&
               !(pl.fused[c].npad == d.npad && pl.fused[c].wide == fused_kind(d) && pl.fused[c].sym == (d.sym != 0) &&
                 pl.fused[c].zd == (d.zd != 0)))
            ++c;
        if (c == pl.fused.size()) {
            FusedClass fc;
            fc.npad = d.npad;
            fc.wide = fused_kind(d);
            fc.sym = d.sym != 0;
            fc.zd = d.zd != 0;
            pl.fused.push_back(fc);
            members.emplace_back();
        }
        members[c].push_back(k);
    }
    for (size_t c = 0; c < pl.fused.size(); ++c) {
        FusedClass& fc = pl.fused[c];
        std::vector<qap::InstDesc> descs;
        std::vector<int2> blkmap;
        const int wpb = qap::fused_particles_per_block(fc.npad, fc.wide, fc.sym, fc.zd);
        for (int k : members[c]) {
            const int j = (int)descs.size();
            descs.push_back(all[(size_t)k]);
            for (int first = 0; first < all[(size_t)k].P; first += wpb) blkmap.push_back(make_int2(j, first));
        }
        fc.blocks = (int)blkmap.size();
        fc.host = descs;
        e = plan_upload(pl, &fc.descs, descs);
        if (e == hipSuccess) e = plan_upload(pl, &fc.blkmap, blkmap);
        if (e != hipSuccess) return dev_err(nullptr, e);
    }
    std::stable_sort(pl.fused.begin(), pl.fused.end(),
                     [](const FusedClass& a, const FusedClass& b) { return a.npad > b.npad; });
    return QAP_OK;
}

// The best-ever record of an instance from its groups' records: the lowest
// goal, first reached (earliest iteration, then lowest swarm) -- the record a
// single chain over all swarms keeps.
qap::BestRec combine_best(const std::vector<qap::BestRec>& r)
{
    qap::BestRec b = r[0];
    for (size_t j = 1; j < r.size(); ++j)
        if (r[j].goal < b.goal || (r[j].goal == b.goal && (r[j].iter < b.iter || (r[j].iter == b.iter && r[j].swarm < b.swarm))))
            b = r[j];
    return b;
}

// Quiesce a handle and release its launch plan: the chains' plans, graphs and
// migration table (streams and events are kept for reuse).
void drop_plan(qap_swarm* h)
{
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (hipStream_t st : h->gstream) (void)hipStreamSynchronize(st);
    for (hipGraphExec_t& g : h->graphs)
        if (g) (void)hipGraphExecDestroy(g), g = nullptr;
    for (hipGraphExec_t& g : h->graphs_k)
        if (g) (void)hipGraphExecDestroy(g), g = nullptr;
    for (StepPlan& pl : h->plans) free_plan(pl);
    h->plans.clear();
    dev_free(h->migr_descs);
    h->migr_descs = nullptr;
    h->migr.clear();
    h->graph_failed = false;
}

// Algorithmic bytes of one iteration of an instance (its weight when whole
// instances are spread over the chains).
double instance_weight(const Instance& I)
{
    return (double)I.P * (8.0 * I.n * I.n + 3.0 * I.n + 24.0);
}

// Put a handle on launch plan c: each instance's swarm groups and their
// chains, one step plan per chain, the streams and events of the chains.
// The instances' per-group best records are first merged into record 0 and
// every group counter set to the instance's iteration, so a plan can change
// between any two steps.
int apply_plan(qap_swarm* h, const PlanCfg& c)
{
    drop_plan(h);
    const int count = (int)h->inst.size();
    for (Instance& I : h->inst) {
        std::vector<qap::BestRec> r((size_t)kMaxChains);
        int t = 0;
        hipError_t e = hipMemcpy(r.data(), I.d.best, sizeof(qap::BestRec) * kMaxChains, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(&t, I.d.iter, sizeof t, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return dev_err(h, e);
        r.resize((size_t)std::max(I.groups, 1));
        std::vector<qap::BestRec> out((size_t)kMaxChains);
        for (qap::BestRec& b : out) {
            std::memset(&b, 0, sizeof b);
            b.goal = LLONG_MAX;
        }
        out[0] = combine_best(r);
        const std::vector<int> ts((size_t)kMaxChains, t);
        e = hipMemcpy(I.d.best, out.data(), sizeof(qap::BestRec) * kMaxChains, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(I.d.iter, ts.data(), sizeof(int) * kMaxChains, hipMemcpyHostToDevice);
        if (e != hipSuccess) return dev_err(h, e);
    }
    // groups and chains
    std::vector<double> load((size_t)c.chains, 0.0);
    std::vector<int> order((size_t)count);
    for (int k = 0; k < count; ++k) order[(size_t)k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return instance_weight(h->inst[(size_t)a]) > instance_weight(h->inst[(size_t)b]);
    });
    for (int k : order) {
        Instance& I = h->inst[(size_t)k];
        const bool fused = h->engine == QAP_ENGINE_FUSED && qap::fused_supported(I.d);
        if (c.split == 0) {
            // an instance whose parameters fix its number of groups keeps it
            const int cap = I.param_groups > 0 ? I.param_groups : c.chains;
            make_groups(I, fused ? std::min({c.chains, I.m, cap}) : 1);
            I.chain.assign((size_t)I.groups, 0);
            for (int j = 0; j < I.groups; ++j) I.chain[(size_t)j] = j;
        } else if (c.split == 1) {
            // whole instances, the heaviest first onto the least loaded chain
            make_groups(I, 1);
            const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            I.chain.assign(1, q);
            load[(size_t)q] += instance_weight(I);
        } else {
            make_groups(I, 1);  // chains assigned per class below
        }
    }
    if (c.split == 2) {
        // whole kernel classes (padded size, contraction kind, symmetry,
        // diagonals; the per-stage instances form one more), the heaviest
        // first onto the least loaded chain: each chain launches few classes
        std::vector<long long> key((size_t)count);
        for (int k = 0; k < count; ++k) {
            const Instance& I = h->inst[(size_t)k];
            const bool fused = h->engine == QAP_ENGINE_FUSED && qap::fused_supported(I.d);
            key[(size_t)k] = fused ? ((long long)I.d.npad << 8) | (fused_kind(I.d) << 4) | (I.d.sym << 1) | I.d.zd : -1;
        }
        std::vector<long long> keys(key);
        std::sort(keys.begin(), keys.end());
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        std::vector<double> weight(keys.size(), 0.0);
        for (int k = 0; k < count; ++k)
            weight[(size_t)(std::lower_bound(keys.begin(), keys.end(), key[(size_t)k]) - keys.begin())] +=
                instance_weight(h->inst[(size_t)k]);
        std::vector<int> cls(keys.size());
        for (size_t i = 0; i < cls.size(); ++i) cls[i] = (int)i;
        std::stable_sort(cls.begin(), cls.end(), [&](int a, int b) { return weight[(size_t)a] > weight[(size_t)b]; });
        std::vector<int> chain_of(keys.size(), 0);
        for (int ci : cls) {
            const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            chain_of[(size_t)ci] = q;
            load[(size_t)q] += weight[(size_t)ci];
        }
        for (int k = 0; k < count; ++k)
            h->inst[(size_t)k].chain.assign(
                1, chain_of[(size_t)(std::lower_bound(keys.begin(), keys.end(), key[(size_t)k]) - keys.begin())]);
    }
    int G = 1;
    for (const Instance& I : h->inst)
        for (int q : I.chain) G = std::max(G, q + 1);
    h->plans.resize((size_t)G);
    for (int q = 0; q < G; ++q) {
        std::vector<qap::InstDesc> descs;
        std::vector<int> own;
        for (int k = 0; k < count; ++k) {
            const Instance& I = h->inst[(size_t)k];
            for (int j = 0; j < I.groups; ++j)
                if (I.chain[(size_t)j] == q) {
                    descs.push_back(I.gdesc[(size_t)j]);
                    own.push_back(k);
                }
        }
        const int rc = build_plan(h, h->plans[(size_t)q], descs, own);
        if (rc != QAP_OK) return rc;
    }
    std::vector<qap::InstDesc> mig;
    for (int k = 0; k < count; ++k) {
        const Instance& I = h->inst[(size_t)k];
        if (I.groups > 1 && I.d.migrate && I.d.migr_d > 0) {
            h->migr.push_back(k);
            mig.push_back(I.d);
        }
    }
    if (!mig.empty()) {
        void* q = nullptr;
        hipError_t e = dev_malloc(&q, sizeof(qap::InstDesc) * mig.size());
        if (e == hipSuccess) e = hipMemcpy(q, mig.data(), sizeof(qap::InstDesc) * mig.size(), hipMemcpyHostToDevice);
        h->migr_descs = static_cast<qap::InstDesc*>(q);
        if (e != hipSuccess) return dev_err(nullptr, e);
    }
    // chain 0 runs on the handle's stream, the others on streams of their own
    // (a process's streams share the runtime's hardware queues, 4 by default:
    // two chains on one queue run one after the other)
    if (h->gstream.empty()) h->gstream.push_back(h->stream);
    while ((int)h->gstream.size() < G) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return QAP_ERR_DEVICE;
        h->gstream.push_back(st);
    }
    while ((int)h->gevent.size() < G) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return QAP_ERR_DEVICE;
        h->gevent.push_back(ev);
    }
    h->graphs.assign((size_t)G, nullptr);
    h->graphs_k.assign((size_t)G, nullptr);
    h->cfg = c;
    return QAP_OK;
}

// The plan a handle starts with: as many chains as the instances' parameters
// ask for (3 when automatic), swarms split over them, graphs of 8 iterations.
PlanCfg default_plan(const qap_swarm* h)
{
    PlanCfg c;
    c.chains = 1;
    for (const Instance& I : h->inst) c.chains = std::max(c.chains, I.param_groups > 0 ? I.param_groups : kStreamGroups);
    c.split = 0;
    c.ipg = kItersPerGraph;
    return c;
}

// ------------------------------------------------------------------ plan cache
// The plans chosen by qap_swarm_tune are kept in a text file named by the
// environment variable QAP_SWARM_TUNE_CACHE, one line per workload signature:
//   <signature> <chains> <split> <iterations per graph> <ms per iteration>
// The signature hashes (FNV-1a, 64 bits) the device's architecture name and
// compute-unit count and, per instance, what the launches depend on: n, the
// swarm layout, the contraction path and kind, the mode and the engine.
std::string plan_signature(const qap_swarm* h)
{
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, h->device);
    std::string key = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "/" +
                      std::to_string(h->engine);
    for (const Instance& I : h->inst) {
        const InstDesc& d = I.d;
        key += ";" + std::to_string(d.n) + "," + std::to_string(d.m) + "," + std::to_string(d.S) + "," +
               std::to_string(d.path) + "," + std::to_string(d.split) + "," + std::to_string(d.sym) + "," +
               std::to_string(d.zd) + "," + std::to_string(d.sx) + "," + std::to_string(d.ls) + "," +
               std::to_string(d.migrate ? d.period : 0) + "," + std::to_string(I.param_groups);
    }
    unsigned long long x = 1469598103934665603ull;
    for (unsigned char ch : key) {
        x ^= ch;
        x *= 1099511628211ull;
    }
    char buf[17];
    std::snprintf(buf, sizeof buf, "%016llx", x);
    return std::string(buf);
}

const char* cache_path() { return std::getenv("QAP_SWARM_TUNE_CACHE"); }

bool valid_plan(const PlanCfg& c)
{
    return c.chains >= 1 && c.chains <= kMaxChains && c.split >= 0 && c.split <= 2 && c.ipg >= 0 &&
           c.ipg <= 64;
}

// The cached plan of this handle's signature, if the cache names one.
bool cached_plan(const qap_swarm* h, PlanCfg* out)
{
    const char* path = cache_path();
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    const std::string sig = plan_signature(h);
    char key[64];
    PlanCfg c;
    float ms = 0.0f;
    bool found = false;
    while (std::fscanf(f, "%63s %d %d %d %f", key, &c.chains, &c.split, &c.ipg, &ms) == 5)
        if (sig == key && valid_plan(c)) {
            *out = c;  // the last line for a signature wins
            found = true;
        }
    std::fclose(f);
    return found;
}

void store_plan(const qap_swarm* h, const PlanCfg& c, float ms)
{
    const char* path = cache_path();
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %.5f\n", plan_signature(h).c_str(), c.chains, c.split, c.ipg, ms);
    std::fclose(f);
}

constexpr int kEvPerIter = 2 * QAP_NUM_STAGES;

// A fresh set of events (ev[2s], ev[2s+1] bracket stage s, see ev_set): its
// index, or -1 if events cannot be created.  Growing the pool may move it, so
// callers keep indices, not pointers, across calls.
long prof_events(qap_swarm* h)
{
    if (h->ev_used + kEvPerIter > h->ev_pool.size()) {
        for (int i = 0; i < kEvPerIter; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            h->ev_pool.push_back(e);
        }
        h->ev_mask.push_back(0);
    }
    const long set = (long)(h->ev_used / kEvPerIter);
    h->ev_mask[(size_t)set] = 0;
    h->ev_used += kEvPerIter;
    return set;
}

hipEvent_t* ev_set(qap_swarm* h, long set) { return h->ev_pool.data() + (size_t)set * kEvPerIter; }

// Fold the recorded event pairs into the per-stage totals.
int prof_collect(qap_swarm* h)
{
    for (hipStream_t st : h->gstream) {
        const hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return dev_err(h, e);
    }
    for (size_t base = 0; base + kEvPerIter <= h->ev_used; base += kEvPerIter) {
        const uint8_t mask = h->ev_mask[base / kEvPerIter];
        for (int s = 0; s < QAP_NUM_STAGES; ++s) {
            float ms = 0.0f;
            if (((mask >> s) & 1) &&
                hipEventElapsedTime(&ms, h->ev_pool[base + 2 * s], h->ev_pool[base + 2 * s + 1]) == hipSuccess)
                h->stage_ms[s] += ms;
        }
    }
    (void)hipGetLastError();
    h->ev_used = 0;
    return QAP_OK;
}

// One iteration of stream group j, launched one by one on its stream: the
// fused classes, the per-stage instances, then the batched bests.  With
// profiling on, events bracket the stages.
int enqueue_iteration(qap_swarm* h, int j)
{
    const StepPlan& pl = h->plans[(size_t)j];
    hipStream_t st = h->gstream[(size_t)j];
    hipError_t e = hipSuccess;
    long set = -1;
    if (h->profiling) {
        if (h->ev_used + kEvPerIter * (1 + pl.plain.size()) > 4096) {
            const int rc = prof_collect(h);
            if (rc != QAP_OK) return rc;
        }
        set = prof_events(h);
        if (set < 0) return dev_err(h, hipErrorOutOfMemory);
    }
#define REC(i)                                                                                     \
    do {                                                                                           \
        if (set >= 0 && (e = hipEventRecord(ev_set(h, set)[i], st)) != hipSuccess) return dev_err(h, e); \
    } while (0)
    if (!pl.fused.empty()) {
        REC(2 * QAP_STAGE_FUSED);
        for (const FusedClass& fc : pl.fused) {
            e = qap::launch_fused_class(fc.npad, fc.wide, fc.sym, fc.zd, fc.host.size() == 1 ? &fc.host[0] : nullptr,
                                        fc.descs, fc.blkmap, fc.blocks, st);
            if (e != hipSuccess) return dev_err(h, e);
        }
        REC(2 * QAP_STAGE_FUSED + 1);
        if (set >= 0) h->ev_mask[(size_t)set] |= 1u << QAP_STAGE_FUSED;
    }
    for (size_t q = 0; q < pl.plain.size(); ++q) {
        const Instance& I = h->inst[(size_t)pl.plain[q]];
        long setp = -1;
        if (h->profiling) {
            setp = prof_events(h);
            if (setp < 0) return dev_err(h, hipErrorOutOfMemory);
        }
        e = qap::launch_plain_step(I.d, I.mul24, h->grid_gd, st, setp >= 0 ? ev_set(h, setp) : nullptr);
        if (e != hipSuccess) return dev_err(h, e);
        if (setp >= 0)
            h->ev_mask[(size_t)setp] |= (1u << QAP_STAGE_SX) | (1u << QAP_STAGE_VELOCITY) | (1u << QAP_STAGE_GOAL_DELTA);
    }
    REC(2 * QAP_STAGE_BESTS);
    e = qap::launch_bests(pl.descs, pl.smap, pl.total_swarms, pl.count, 0, st);
    if (e != hipSuccess) return dev_err(h, e);
    REC(2 * QAP_STAGE_BESTS + 1);
    if (set >= 0) h->ev_mask[(size_t)set] |= 1u << QAP_STAGE_BESTS;
#undef REC
    return QAP_OK;
}

// Capture `iters` iterations of group j into a graph (replayed once per
// `iters` iterations).  A stream that cannot be captured leaves the handle on
// eager launches.
void capture_iterations(qap_swarm* h, int j, int iters, hipGraphExec_t* out)
{
    hipStream_t st = h->gstream[(size_t)j];
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        h->graph_failed = true;
        return;
    }
    int rc = QAP_OK;
    for (int i = 0; i < iters && rc == QAP_OK; ++i) rc = enqueue_iteration(h, j);
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != QAP_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        if (rc != QAP_OK) h->sticky = QAP_OK;  // nothing ran: the capture only recorded
        h->graph_failed = true;
        return;
    }
    if (hipGraphInstantiate(out, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        h->graph_failed = true;
    }
    (void)hipGraphDestroy(g);
}

// Whether Alg. 2 of an instance stepped in several groups falls due after
// any of the iterations it + 1 .. it + count of this step call.
bool migration_due(const qap_swarm* h, int it, int count)
{
    for (int k : h->migr) {
        const Instance& I = h->inst[(size_t)k];
        for (int c = 1; c <= count; ++c)
            if ((I.t + it + c) % I.d.period == 0) return true;
    }
    return false;
}

int get_instance(qap_swarm* h, int32_t k, Instance** out)
{
    if (!h) return QAP_ERR_INVALID_ARG;
    if (h->sticky != QAP_OK) return h->sticky;
    if (k < 0 || k >= (int)h->inst.size()) return QAP_ERR_INVALID_ARG;
    *out = &h->inst[(size_t)k];
    return QAP_OK;
}

}  // namespace

extern "C" {

const char* qap_swarm_strerror(int code)
{
    switch (code) {
    case QAP_OK: return "ok";
    case QAP_ERR_INVALID_ARG: return "invalid argument";
    case QAP_ERR_RANGE: return "value range of F or D too wide for an exact contraction path";
    case QAP_ERR_NOMEM: return "out of memory";
    case QAP_ERR_DEVICE: return "device error";
    case QAP_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown error";
    }
}

void qap_swarm_destroy(qap_swarm* h)
{
    if (!h) return;
    for (hipStream_t st : h->gstream) (void)hipStreamSynchronize(st);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (hipGraphExec_t g : h->graphs)
        if (g) (void)hipGraphExecDestroy(g);
    for (hipGraphExec_t g : h->graphs_k)
        if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->gevent) (void)hipEventDestroy(e);
    for (size_t j = 1; j < h->gstream.size(); ++j) (void)hipStreamDestroy(h->gstream[j]);
    free_plan(h->init);
    for (StepPlan& pl : h->plans) free_plan(pl);
    dev_free(h->migr_descs);
    for (Instance& I : h->inst) free_instance(I);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

}  // extern "C"

namespace {

// *hold keeps the handle while it is being built, so that the entry point can
// release it if a host allocation throws; it is cleared on every other failure
// (the handle is released here).
int impl_init_batch(const qap_instance* insts, const qap_params* prms, int32_t count, qap_swarm** out,
                    qap_swarm** hold)
{
    if (!out) return QAP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!insts || !prms || count < 1) return QAP_ERR_INVALID_ARG;
    // every host-side check comes before the first HIP call
    std::vector<int> path((size_t)count), sym((size_t)count), mul24((size_t)count), zd((size_t)count),
        split((size_t)count);
    for (int k = 0; k < count; ++k) {
        int rc = check_params(&insts[k], &prms[k]);
        if (rc != QAP_OK) return rc;
        if (prms[k].engine != prms[0].engine) return QAP_ERR_INVALID_ARG;
        rc = choose_path(&insts[k], &prms[k], prms[0].engine, &path[(size_t)k], &sym[(size_t)k], &mul24[(size_t)k],
                         &zd[(size_t)k], &split[(size_t)k]);
        if (rc != QAP_OK) return rc;
    }
    qap_swarm* h = new (std::nothrow) qap_swarm();
    if (!h) return QAP_ERR_NOMEM;
    *hold = h;
    const auto fail = [&](int rc) {
        qap_swarm_destroy(h);
        *hold = nullptr;
        return rc;
    };
    h->engine = prms[0].engine;
    if (hipGetDevice(&h->device) != hipSuccess) return fail(QAP_ERR_DEVICE);
    if (scratch_address(h->device, &h->scratch) != hipSuccess) return fail(QAP_ERR_DEVICE);
    if (prms[0].stream) {
        h->stream = (hipStream_t)prms[0].stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return fail(QAP_ERR_DEVICE);
        h->own_stream = true;
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
    h->grid_gd = std::max(64, cus * 8);
    h->inst.resize((size_t)count);
    for (int k = 0; k < count; ++k) {
        const int rc = setup_instance(h, h->inst[(size_t)k], &insts[k], &prms[k], path[(size_t)k], sym[(size_t)k],
                                      mul24[(size_t)k], zd[(size_t)k], split[(size_t)k]);
        if (rc != QAP_OK) return fail(rc);
    }
    // the whole-instance plan (iteration 0), then the launch plan
    std::vector<qap::InstDesc> whole;
    std::vector<int> owner;
    for (int k = 0; k < count; ++k) {
        whole.push_back(h->inst[(size_t)k].d);
        owner.push_back(k);
    }
    int rc = build_plan(h, h->init, whole, owner);
    if (rc == QAP_OK) {
        PlanCfg c = default_plan(h);
        (void)cached_plan(h, &c);
        rc = apply_plan(h, c);
    }
    if (rc == QAP_OK) {
        hipError_t e = qap::launch_bests(h->init.descs, h->init.smap, h->init.total_swarms, count, 1, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        rc = dev_err(nullptr, e);
    }
    if (rc != QAP_OK) return fail(rc);
    *hold = nullptr;
    *out = h;
    return QAP_OK;
}

int impl_step(qap_swarm* h, int32_t iterations)
{
    if (!h || iterations < 0) return QAP_ERR_INVALID_ARG;
    if (h->sticky != QAP_OK) return h->sticky;
    if (iterations == 0) return QAP_OK;
    const int G = (int)h->plans.size();
    hipError_t e = hipSuccess;
    // the groups start after the work already on the handle's stream ...
    auto fork = [&]() {
        hipError_t r = hipEventRecord(h->gevent[0], h->stream);
        for (int j = 1; j < G && r == hipSuccess; ++j) r = hipStreamWaitEvent(h->gstream[(size_t)j], h->gevent[0], 0);
        return r;
    };
    auto join = [&]() {
        hipError_t r = hipSuccess;
        for (int j = 1; j < G && r == hipSuccess; ++j) {
            r = hipEventRecord(h->gevent[(size_t)j], h->gstream[(size_t)j]);
            if (r == hipSuccess) r = hipStreamWaitEvent(h->stream, h->gevent[(size_t)j], 0);
        }
        return r;
    };
    if (G > 1) {
        e = fork();
        if (e != hipSuccess) return dev_err(h, e);
    }
    for (int it = 0; it < iterations;) {
        // a graph of several iterations where no migration join falls inside it
        const int K = h->cfg.ipg;
        const bool graphs = !h->profiling && K > 0 && !h->graph_failed;
        bool record = false;  // some instance records its statistics after every iteration
        for (const Instance& I : h->inst) record = record || I.hist_cap > 0;
        const bool multi = graphs && K > 1 && iterations - it >= K && !migration_due(h, it, K) && !record;
        const int chunk = multi ? K : 1;
        for (int j = 0; j < G; ++j) {
            hipGraphExec_t* gx = multi ? &h->graphs_k[(size_t)j] : &h->graphs[(size_t)j];
            if (graphs && !*gx) capture_iterations(h, j, chunk, gx);
            if (graphs && *gx) {
                e = hipGraphLaunch(*gx, h->gstream[(size_t)j]);
                if (e != hipSuccess) return dev_err(h, e);
                continue;
            }
            for (int c = 0; c < chunk; ++c) {
                const int rc = enqueue_iteration(h, j);
                if (rc != QAP_OK) return rc;
            }
        }
        if (h->profiling) h->prof_iters += chunk;
        // Alg. 2 of the instances stepped in several groups, when due (only
        // after single iterations): the groups join, one launch migrates, and
        // they fork again before the next iteration reads P^G
        // and the per-iteration statistics of the recording instances (on
        // the handle's stream, once every chain finished the iteration; no
        // host synchronisation)
        const bool mig = !multi && migration_due(h, it, 1);
        if (mig || record) {
            if (G > 1) e = join();
            if (e == hipSuccess && mig) e = qap::launch_migrate(h->migr_descs, (int)h->migr.size(), h->stream);
            for (size_t k = 0; k < h->inst.size() && e == hipSuccess && record; ++k) {
                const Instance& I = h->inst[k];
                if (I.hist_cap > 0)
                    e = qap::launch_history(I.d.goal, I.d.iter, I.m, I.S, I.hist_nq, I.hist_ranks, I.hist_bins,
                                            I.hist_lo, I.hist_hi, I.hist_cap, I.ring_t, I.ring_q, I.ring_h,
                                            h->stream);
            }
            if (e == hipSuccess && G > 1) e = fork();
            if (e != hipSuccess) return dev_err(h, e);
        }
        it += chunk;
    }
    for (Instance& I : h->inst) {
        I.stepped = true;
        I.t += iterations;
    }
    // ... and the handle's stream continues after all of them
    if (G > 1) e = join();
    return dev_err(h, e);
}

int impl_sync(qap_swarm* h)
{
    if (!h) return QAP_ERR_INVALID_ARG;
    if (h->sticky != QAP_OK) return h->sticky;
    return dev_err(h, hipStreamSynchronize(h->stream));
}

// The instance's best-ever record (its groups' records combined); waits.
hipError_t read_best(qap_swarm* h, const Instance& I, qap::BestRec* out)
{
    std::vector<qap::BestRec> r((size_t)I.groups);
    hipError_t e = hipMemcpyAsync(r.data(), I.d.best, sizeof(qap::BestRec) * I.groups, hipMemcpyDeviceToHost,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) *out = combine_best(r);
    return e;
}

int impl_best(qap_swarm* h, int32_t instance, int64_t* goal, int32_t* perm, int32_t* iter_found)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    qap::BestRec br;
    const hipError_t e = read_best(h, *I, &br);
    if (e != hipSuccess) return dev_err(h, e);
    if (goal) *goal = br.goal;
    if (iter_found) *iter_found = br.iter;
    if (perm)
        for (int j = 0; j < I->n; ++j) perm[j] = br.perm[j];
    return QAP_OK;
}

int impl_swarm_bests(qap_swarm* h, int32_t instance, int64_t* goals)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (!goals) return QAP_ERR_INVALID_ARG;
    hipError_t e = hipMemcpyAsync(goals, I->d.goalPG, sizeof(long long) * I->m, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return dev_err(h, e);
}

int impl_get_state(qap_swarm* h, int32_t instance, qap_state* st)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (!st) return QAP_ERR_INVALID_ARG;
    const InstDesc& d = I->d;
    hipError_t e = hipStreamSynchronize(h->stream);
    int t = 0;
    if (e == hipSuccess) e = hipMemcpy(&t, d.iter, sizeof t, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_err(h, e);
    const int cur = t & 1;
    const size_t n = (size_t)I->n, P = (size_t)I->P, m = (size_t)I->m;
    std::vector<uint8_t> buf(std::max(P, m) * n);
    auto perms_out = [&](const uint8_t* src, size_t rows, int32_t* dst) -> hipError_t {
        hipError_t ee = hipMemcpy(buf.data(), src, rows * n, hipMemcpyDeviceToHost);
        if (ee == hipSuccess)
            for (size_t i = 0; i < rows * n; ++i) dst[i] = buf[i];
        return ee;
    };
    if (e == hipSuccess && st->V) {
        // V = fl(U * scale) per column, the value every kernel reads
        std::vector<float> sc(P * n);
        e = hipMemcpy(st->V, d.V[cur], P * n * n * sizeof(float), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(sc.data(), d.Vinv[cur], P * n * sizeof(float), hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            for (size_t k = 0; k < P; ++k)
                for (size_t r = 0; r < n; ++r)
                    for (size_t c = 0; c < n; ++c) {
                        volatile float prod = st->V[(k * n + r) * n + c] * sc[k * n + c];
                        st->V[(k * n + r) * n + c] = prod;
                    }
    }
    if (e == hipSuccess && st->X) e = perms_out(d.X[cur], P, st->X);
    if (e == hipSuccess && st->PL) e = perms_out(d.PL, P, st->PL);
    if (e == hipSuccess && st->goal) e = hipMemcpy(st->goal, d.goal, P * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && st->goalPL) e = hipMemcpy(st->goalPL, d.goalPL, P * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && st->PG) e = perms_out(d.PG, m, st->PG);
    if (e == hipSuccess && st->goalPG) e = hipMemcpy(st->goalPG, d.goalPG, m * 8, hipMemcpyDeviceToHost);
    qap::BestRec br;
    if (e == hipSuccess) e = read_best(h, *I, &br);
    if (e != hipSuccess) return dev_err(h, e);
    st->best_goal = br.goal;
    st->best_iter = br.iter;
    st->best_swarm = br.swarm;
    st->best_particle = br.member;
    if (st->best_perm)
        for (size_t j = 0; j < n; ++j) st->best_perm[j] = br.perm[j];
    st->iteration = t;
    return QAP_OK;
}

int impl_set_state(qap_swarm* h, int32_t instance, const qap_state* st)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (!st || !st->V || !st->X || !st->PL || !st->goal || !st->goalPL || !st->PG || !st->goalPG ||
        !st->best_perm || st->iteration < 0)
        return QAP_ERR_INVALID_ARG;
    const InstDesc& d = I->d;
    const size_t n = (size_t)I->n, P = (size_t)I->P, m = (size_t)I->m;
    auto valid = [&](const int32_t* p, size_t rows) {
        std::vector<char> seen(n);
        for (size_t r = 0; r < rows; ++r) {
            std::fill(seen.begin(), seen.end(), 0);
            for (size_t j = 0; j < n; ++j) {
                const int32_t v = p[r * n + j];
                if (v < 0 || (size_t)v >= n || seen[(size_t)v]) return false;
                seen[(size_t)v] = 1;
            }
        }
        return true;
    };
    if (!valid(st->X, P) || !valid(st->PL, P) || !valid(st->PG, m) || !valid(st->best_perm, 1))
        return QAP_ERR_INVALID_ARG;
    hipError_t e = hipStreamSynchronize(h->stream);
    const int t = st->iteration, cur = t & 1;
    std::vector<uint8_t> buf(std::max(P, m) * n);
    auto perms_in = [&](const int32_t* src, size_t rows, uint8_t* dst) -> hipError_t {
        for (size_t i = 0; i < rows * n; ++i) buf[i] = (uint8_t)src[i];
        return hipMemcpy(dst, buf.data(), rows * n, hipMemcpyHostToDevice);
    };
    if (e == hipSuccess)
        e = hipMemcpy(d.V[cur], st->V, P * n * n * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const std::vector<float> ones(P * n, 1.0f);
        e = hipMemcpy(d.Vinv[cur], ones.data(), P * n * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = perms_in(st->X, P, d.X[cur]);
    if (e == hipSuccess) e = perms_in(st->PL, P, d.PL);
    if (e == hipSuccess) e = hipMemcpy(d.goal, st->goal, P * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.goalPL, st->goalPL, P * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = perms_in(st->PG, m, d.PG);
    if (e == hipSuccess) e = hipMemcpy(d.goalPG, st->goalPG, m * 8, hipMemcpyHostToDevice);
    // the record goes to group 0, the other groups' records start empty
    std::vector<qap::BestRec> recs((size_t)kMaxChains);
    for (qap::BestRec& r : recs) {
        std::memset(&r, 0, sizeof r);
        r.goal = LLONG_MAX;
    }
    recs[0].goal = st->best_goal;
    recs[0].iter = st->best_iter;
    recs[0].swarm = st->best_swarm;
    recs[0].member = st->best_particle;
    for (size_t j = 0; j < n; ++j) recs[0].perm[j] = (uint8_t)st->best_perm[j];
    const std::vector<int> ts((size_t)kMaxChains, t);
    if (e == hipSuccess) e = hipMemcpy(d.best, recs.data(), sizeof(qap::BestRec) * kMaxChains, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.iter, ts.data(), sizeof(int) * kMaxChains, hipMemcpyHostToDevice);
    I->stepped = false;  // the previous-state buffers no longer belong to this state
    I->t = t;
    return dev_err(h, e);
}

int impl_eval(qap_swarm* h, int32_t instance, const int32_t* perms, int32_t count, int64_t* goals,
                   int64_t* deltas)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (!perms || !goals || count < 0) return QAP_ERR_INVALID_ARG;
    if (count == 0) return QAP_OK;
    const size_t n = (size_t)I->n;
    std::vector<uint8_t> hp((size_t)count * n);
    std::vector<char> seen(n);
    for (int r = 0; r < count; ++r) {
        std::fill(seen.begin(), seen.end(), 0);
        for (size_t j = 0; j < n; ++j) {
            const int32_t v = perms[(size_t)r * n + j];
            if (v < 0 || (size_t)v >= n || seen[(size_t)v]) return QAP_ERR_INVALID_ARG;
            seen[(size_t)v] = 1;
            hp[(size_t)r * n + j] = (uint8_t)v;
        }
    }
    uint8_t* dp = nullptr;
    long long* dg = nullptr;
    long long* dd = nullptr;
    hipError_t e = dev_malloc(reinterpret_cast<void**>(&dp), hp.size());
    if (e == hipSuccess) e = dev_malloc(reinterpret_cast<void**>(&dg), sizeof(long long) * (size_t)count);
    if (e == hipSuccess && deltas) e = dev_malloc(reinterpret_cast<void**>(&dd), sizeof(long long) * (size_t)count * n * n);
    if (e == hipSuccess) e = hipMemcpyAsync(dp, hp.data(), hp.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        if (qap::fused_supported(I->d))
            e = qap::launch_eval_mfma(I->d, dp, count, dg, dd, h->stream);
        else
            e = qap::launch_goal_delta_i32(I->d, I->mul24, h->grid_gd, dp, count, 1, dg, dd, h->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(goals, dg, sizeof(long long) * (size_t)count, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && deltas)
        e = hipMemcpyAsync(deltas, dd, sizeof(long long) * (size_t)count * n * n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    dev_free(dp);
    dev_free(dg);
    dev_free(dd);
    return dev_err(h, e);
}

int impl_deltas(qap_swarm* h, int32_t instance, int32_t particle, int64_t* out, int32_t* perm)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (!out || particle < 0 || particle >= I->P || !I->stepped) return QAP_ERR_INVALID_ARG;
    const size_t n = (size_t)I->n;
    int t = 0;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(&t, I->d.iter, sizeof t, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_err(h, e);
    if (t < 1) return QAP_ERR_INVALID_ARG;
    uint8_t* dp = nullptr;
    long long* dg = nullptr;
    long long* dd = nullptr;
    e = dev_malloc(reinterpret_cast<void**>(&dp), n);
    if (e == hipSuccess) e = dev_malloc(reinterpret_cast<void**>(&dg), sizeof(long long));
    if (e == hipSuccess) e = dev_malloc(reinterpret_cast<void**>(&dd), sizeof(long long) * n * n);
    // the S_x output of the step t - 1 -> t, then its goal and deltas on the
    // instance's contraction path
    if (e == hipSuccess) e = qap::launch_sx_probe(I->d, particle, t - 1, dp, h->stream);
    if (e == hipSuccess) {
        if (qap::fused_supported(I->d))
            e = qap::launch_eval_mfma(I->d, dp, 1, dg, dd, h->stream);
        else
            e = qap::launch_goal_delta_i32(I->d, I->mul24, h->grid_gd, dp, 1, 1, dg, dd, h->stream);
    }
    std::vector<uint8_t> hp(n);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dd, sizeof(long long) * n * n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), dp, n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    dev_free(dp);
    dev_free(dg);
    dev_free(dd);
    if (e != hipSuccess) return dev_err(h, e);
    if (perm)
        for (size_t j = 0; j < n; ++j) perm[j] = hp[j];
    return QAP_OK;
}

int impl_profile(qap_swarm* h, int32_t enable, double* stage_ms, int64_t* launches)
{
    if (!h || (enable != 0 && enable != 1)) return QAP_ERR_INVALID_ARG;
    if (h->sticky != QAP_OK) return h->sticky;
    if (h->profiling) {
        const int rc = prof_collect(h);
        if (rc != QAP_OK) return rc;
    }
    if (stage_ms)
        for (int s = 0; s < QAP_NUM_STAGES; ++s) stage_ms[s] = h->stage_ms[s];
    if (launches) *launches = h->prof_iters;
    if ((bool)enable != h->profiling) {
        h->profiling = enable != 0;
        for (double& v : h->stage_ms) v = 0.0;
        h->prof_iters = 0;
    }
    return QAP_OK;
}

int impl_stats(qap_swarm* h, int32_t instance, int32_t nq, const int32_t* q_ppm, int64_t* swarm_q,
                    int64_t* pop_q, int32_t bins, int64_t lo, int64_t hi, int64_t* swarm_hist, int64_t* pop_hist)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (nq < 0 || nq > QAP_STATS_MAX_RANKS || (nq > 0 && !q_ppm)) return QAP_ERR_INVALID_ARG;
    for (int j = 0; j < nq; ++j)
        if (q_ppm[j] < 1 || q_ppm[j] > 1000000) return QAP_ERR_INVALID_ARG;
    if (bins < 0 || bins > QAP_STATS_MAX_BINS) return QAP_ERR_INVALID_ARG;
    if (bins > 0 && (!(lo < hi) || (unsigned long long)hi - (unsigned long long)lo > (1ull << 62) / (unsigned)bins))
        return QAP_ERR_INVALID_ARG;
    const int m = I->m, S = I->S, P = I->P;
    const bool want_q = nq > 0 && (swarm_q || pop_q), want_h = bins > 0 && (swarm_hist || pop_hist);
    if (!want_q && !want_h) return QAP_OK;
    // segments: the m swarms, then the whole population
    std::vector<int> off((size_t)m + 3);
    for (int g = 0; g <= m; ++g) off[(size_t)g] = g * S;
    off[(size_t)m + 1] = 0;
    off[(size_t)m + 2] = P;
    const int nr = std::max(nq, 1);
    std::vector<long long> ranks((size_t)(m + 1) * nr, 1);
    for (int j = 0; j < nq; ++j) {
        const auto rank = [&](long long N) { return std::max(1LL, ((long long)q_ppm[j] * N + 999999) / 1000000); };
        for (int g = 0; g < m; ++g) ranks[(size_t)g * nr + j] = rank(S);
        ranks[(size_t)m * nr + j] = rank(P);
    }
    const size_t b_off = off.size() * sizeof(int), b_rank = ranks.size() * sizeof(long long);
    const size_t b_out = ranks.size() * sizeof(long long), b_hist = (size_t)m * std::max(bins, 1) * 8;
    char* buf = nullptr;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = dev_malloc(reinterpret_cast<void**>(&buf), b_off + b_rank + b_out + b_hist);
    if (e != hipSuccess) return dev_err(h, e);
    int* d_off = (int*)buf;
    long long* d_rank = (long long*)(buf + b_off);
    long long* d_out = (long long*)(buf + b_off + b_rank);
    unsigned long long* d_hist = (unsigned long long*)(buf + b_off + b_rank + b_out);
    std::vector<long long> outq(ranks.size());
    std::vector<unsigned long long> hist((size_t)m * std::max(bins, 1));
    e = hipMemcpy(d_off, off.data(), b_off, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_rank, ranks.data(), b_rank, hipMemcpyHostToDevice);
    if (e == hipSuccess && want_q) e = qap::launch_select(I->d.goal, d_off, m, d_rank, nr, d_out, h->stream);
    if (e == hipSuccess && want_q)
        e = qap::launch_select(I->d.goal, d_off + m + 1, 1, d_rank + (size_t)m * nr, nr, d_out + (size_t)m * nr,
                               h->stream);
    if (e == hipSuccess && want_h) e = qap::launch_hist(I->d.goal, d_off, m, bins, lo, hi, d_hist, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess && want_q) e = hipMemcpy(outq.data(), d_out, b_out, hipMemcpyDeviceToHost);
    if (e == hipSuccess && want_h) e = hipMemcpy(hist.data(), d_hist, b_hist, hipMemcpyDeviceToHost);
    dev_free(buf);
    if (e != hipSuccess) return dev_err(h, e);
    for (int j = 0; j < nq; ++j) {
        if (swarm_q)
            for (int g = 0; g < m; ++g) swarm_q[(size_t)g * nq + j] = outq[(size_t)g * nr + j];
        if (pop_q) pop_q[j] = outq[(size_t)m * nr + j];
    }
    if (want_h) {
        if (pop_hist)
            for (int i = 0; i < bins; ++i) pop_hist[i] = 0;
        for (int g = 0; g < m; ++g)
            for (int i = 0; i < bins; ++i) {
                const long long c = (long long)hist[(size_t)g * bins + i];
                if (swarm_hist) swarm_hist[(size_t)g * bins + i] = c;
                if (pop_hist) pop_hist[i] += c;
            }
    }
    return QAP_OK;
}

// qap_swarm_stats with its scratch in the fixed device array: the request's
// segment offsets and ranks are written by a kernel, the selections and bin
// counts land in the array, and the results are copied from it into the
// caller's arrays.  No allocation, device or host.
int impl_stats_noalloc(qap_swarm* h, int32_t instance, int32_t nq, const int32_t* q_ppm, int64_t* swarm_q,
                       int64_t* pop_q, int32_t bins, int64_t lo, int64_t hi, int64_t* swarm_hist, int64_t* pop_hist)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (nq < 0 || nq > QAP_STATS_MAX_RANKS || (nq > 0 && !q_ppm)) return QAP_ERR_INVALID_ARG;
    for (int j = 0; j < nq; ++j)
        if (q_ppm[j] < 1 || q_ppm[j] > 1000000) return QAP_ERR_INVALID_ARG;
    if (bins < 0 || bins > QAP_STATS_MAX_BINS) return QAP_ERR_INVALID_ARG;
    if (bins > 0 && (!(lo < hi) || (unsigned long long)hi - (unsigned long long)lo > (1ull << 62) / (unsigned)bins))
        return QAP_ERR_INVALID_ARG;
    const bool want_q = nq > 0 && (swarm_q || pop_q), want_h = bins > 0 && (swarm_hist || pop_hist);
    if (!want_q && !want_h) return QAP_OK;
    if (!h->scratch) return QAP_ERR_DEVICE;
    const int m = I->m, S = I->S, P = I->P;
    const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_off = up(sizeof(int) * (size_t)(m + 3));
    const size_t b_rank = up(sizeof(long long) * (size_t)(m + 1) * (size_t)std::max(nq, 1));
    const size_t b_hist = up(sizeof(long long) * (size_t)(m + 1) * (size_t)std::max(bins, 1));
    if (b_off + 2 * b_rank + b_hist > kScratchBytes) return QAP_ERR_UNSUPPORTED;
    char* base = static_cast<char*>(h->scratch);
    int* d_off = reinterpret_cast<int*>(base);
    long long* d_rank = reinterpret_cast<long long*>(base + b_off);
    long long* d_out = reinterpret_cast<long long*>(base + b_off + b_rank);
    unsigned long long* d_hist = reinterpret_cast<unsigned long long*>(base + b_off + 2 * b_rank);
    qap::StatsRanks qr{};
    for (int j = 0; j < nq; ++j) qr.ppm[j] = q_ppm[j];
    hipStream_t st = h->stream;
    const long long* goals = I->d.goal;
    hipError_t e = qap::launch_stats_setup(d_off, d_rank, m, S, P, want_q ? nq : 0, qr, st);
    if (e == hipSuccess && want_q) e = qap::launch_select(goals, d_off, m, d_rank, nq, d_out, st);
    if (e == hipSuccess && want_q)
        e = qap::launch_select(goals, d_off + m + 1, 1, d_rank + (size_t)m * nq, nq, d_out + (size_t)m * nq, st);
    if (e == hipSuccess && want_h) e = qap::launch_hist(goals, d_off, m, bins, lo, hi, d_hist, st);
    if (e == hipSuccess && want_h)
        e = qap::launch_hist(goals, d_off + m + 1, 1, bins, lo, hi, d_hist + (size_t)m * bins, st);
    // nq >= 1 here, so the selections are [m + 1][nq] in the caller's order;
    // counts are below 2^63, so the unsigned words are the int64 values
    if (e == hipSuccess && want_q && swarm_q)
        e = hipMemcpyAsync(swarm_q, d_out, sizeof(long long) * (size_t)m * nq, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && want_q && pop_q)
        e = hipMemcpyAsync(pop_q, d_out + (size_t)m * nq, sizeof(long long) * (size_t)nq, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && want_h && swarm_hist)
        e = hipMemcpyAsync(swarm_hist, d_hist, sizeof(long long) * (size_t)m * bins, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && want_h && pop_hist)
        e = hipMemcpyAsync(pop_hist, d_hist + (size_t)m * bins, sizeof(long long) * (size_t)bins,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return dev_err(h, e);
}

int impl_history_start(qap_swarm* h, int32_t instance, int32_t capacity, int32_t nq, const int32_t* q_ppm,
                       int32_t bins, int64_t lo, int64_t hi)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (capacity < 1 || capacity > QAP_HISTORY_MAX_RECORDS) return QAP_ERR_INVALID_ARG;
    if (nq < 0 || nq > QAP_STATS_MAX_RANKS || (nq > 0 && !q_ppm)) return QAP_ERR_INVALID_ARG;
    for (int j = 0; j < nq; ++j)
        if (q_ppm[j] < 1 || q_ppm[j] > 1000000) return QAP_ERR_INVALID_ARG;
    if (bins < 0 || bins > QAP_STATS_MAX_BINS || (nq == 0 && bins == 0)) return QAP_ERR_INVALID_ARG;
    if (bins > 0 && (!(lo < hi) || (unsigned long long)hi - (unsigned long long)lo > (1ull << 62) / (unsigned)bins))
        return QAP_ERR_INVALID_ARG;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_err(h, e);
    free_history(*I);
    const int m = I->m;
    std::vector<long long> ranks((size_t)(m + 1) * std::max(nq, 1), 1);
    for (int g = 0; g <= m; ++g)
        for (int j = 0; j < nq; ++j) {
            const long long N = g < m ? I->S : I->P;
            ranks[(size_t)g * nq + j] = std::max(1LL, ((long long)q_ppm[j] * N + 999999) / 1000000);
        }
    const size_t cap = (size_t)capacity;
    e = dev_malloc(reinterpret_cast<void**>(&I->hist_ranks), sizeof(long long) * ranks.size());
    if (e == hipSuccess) e = dev_malloc(reinterpret_cast<void**>(&I->ring_t), sizeof(int) * cap);
    if (e == hipSuccess)
        e = dev_malloc(reinterpret_cast<void**>(&I->ring_q), sizeof(long long) * cap * (m + 1) * std::max(nq, 1));
    if (e == hipSuccess)
        e = dev_malloc(reinterpret_cast<void**>(&I->ring_h), sizeof(long long) * cap * (m + 1) * std::max(bins, 1));
    if (e == hipSuccess) e = hipMemcpy(I->hist_ranks, ranks.data(), sizeof(long long) * ranks.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(I->ring_t, 0, sizeof(int) * cap);
    if (e != hipSuccess) {
        free_history(*I);
        return dev_err(h, e);
    }
    I->hist_cap = capacity;
    I->hist_nq = nq;
    I->hist_bins = bins;
    I->hist_lo = lo;
    I->hist_hi = hi;
    I->hist_t0 = I->t;
    return QAP_OK;
}

int impl_history_stop(qap_swarm* h, int32_t instance)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    hipError_t e = hipStreamSynchronize(h->stream);
    free_history(*I);
    return dev_err(h, e);
}

int impl_history_read(qap_swarm* h, int32_t instance, int32_t max_records, int32_t* count, int32_t* iters,
                      int64_t* swarm_q, int64_t* pop_q, int64_t* swarm_hist, int64_t* pop_hist)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (!count || max_records < 0) return QAP_ERR_INVALID_ARG;
    *count = 0;
    if (I->hist_cap == 0) return QAP_ERR_INVALID_ARG;  // not recording
    const int m = I->m, nq = I->hist_nq, bins = I->hist_bins, cap = I->hist_cap;
    const long long recorded = std::min<long long>(I->t - I->hist_t0, cap);
    const int want = (int)std::min<long long>(recorded, max_records);
    if (want == 0) return QAP_OK;
    const size_t rq = (size_t)(m + 1) * std::max(nq, 1), rh = (size_t)(m + 1) * std::max(bins, 1);
    std::vector<int> rt((size_t)cap);
    std::vector<long long> q((size_t)cap * rq);
    std::vector<unsigned long long> hh((size_t)cap * rh);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(rt.data(), I->ring_t, sizeof(int) * cap, hipMemcpyDeviceToHost);
    if (e == hipSuccess && nq > 0) e = hipMemcpy(q.data(), I->ring_q, sizeof(long long) * q.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess && bins > 0) e = hipMemcpy(hh.data(), I->ring_h, sizeof(long long) * hh.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_err(h, e);
    // the latest `want` iterations, oldest first: iteration t sits in slot (t - 1) % cap
    for (int r = 0; r < want; ++r) {
        const long long t = I->t - want + 1 + r;
        const size_t slot = (size_t)((t - 1) % cap);
        if (rt[slot] != (int)t) return QAP_ERR_DEVICE;  // a record that was not written
        if (iters) iters[r] = (int32_t)t;
        for (int g = 0; g < m; ++g) {
            for (int j = 0; j < nq && swarm_q; ++j) swarm_q[((size_t)r * m + g) * nq + j] = q[slot * rq + (size_t)g * nq + j];
            for (int b = 0; b < bins && swarm_hist; ++b)
                swarm_hist[((size_t)r * m + g) * bins + b] = (int64_t)hh[slot * rh + (size_t)g * bins + b];
        }
        for (int j = 0; j < nq && pop_q; ++j) pop_q[(size_t)r * nq + j] = q[slot * rq + (size_t)m * nq + j];
        for (int b = 0; b < bins && pop_hist; ++b) pop_hist[(size_t)r * bins + b] = (int64_t)hh[slot * rh + (size_t)m * bins + b];
    }
    *count = want;
    return QAP_OK;
}

int impl_graph(qap_swarm* h, int32_t* active, int32_t* streams)
{
    if (!h) return QAP_ERR_INVALID_ARG;
    bool all = !h->graphs.empty() && h->cfg.ipg > 0 && !h->graph_failed;
    for (hipGraphExec_t g : h->graphs) all = all && g != nullptr;
    if (active) *active = (all && !h->profiling) ? 1 : 0;
    if (streams) *streams = (int32_t)h->plans.size();
    return QAP_OK;
}

int impl_get_plan(qap_swarm* h, qap_plan* plan)
{
    if (!h || !plan) return QAP_ERR_INVALID_ARG;
    if (h->sticky != QAP_OK) return h->sticky;
    plan->stream_chains = h->cfg.chains;
    plan->split = h->cfg.split;
    plan->iters_per_graph = h->cfg.ipg;
    plan->ms_per_iteration = 0.0f;
    return QAP_OK;
}

int impl_set_plan(qap_swarm* h, const qap_plan* plan)
{
    if (!h || !plan) return QAP_ERR_INVALID_ARG;
    if (h->sticky != QAP_OK) return h->sticky;
    PlanCfg c;
    c.chains = plan->stream_chains;
    c.split = plan->split;
    c.ipg = plan->iters_per_graph;
    if (!valid_plan(c)) return QAP_ERR_INVALID_ARG;
    return apply_plan(h, c);
}

// The state init made, re-created from the seed (every instance at
// iteration 0, then the initial bests); waits.
int reset_state(qap_swarm* h)
{
    int rc = QAP_OK;
    for (Instance& I : h->inst)
        if (rc == QAP_OK) rc = init_state(h, I);
    if (rc != QAP_OK) return rc;
    hipError_t e = qap::launch_bests(h->init.descs, h->init.smap, h->init.total_swarms, (int)h->inst.size(), 1,
                                     h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return dev_err(h, e);
}

constexpr int kTuneWarmup = 10;
constexpr size_t kTuneFinalists = 4;  // plans timed again by the tuner

// Time every candidate plan on the handle's own work (from iteration 0, a
// warm-up, then `trial` iterations between events on the handle's stream),
// keep the fastest, and put the handle back to iteration 0 (the
// initialisation is a function of the seed, so the state is exactly the one
// init made).
int impl_tune(qap_swarm* h, int32_t trial, qap_plan* chosen)
{
    if (!h || trial < 1 || trial > 4096) return QAP_ERR_INVALID_ARG;
    if (h->sticky != QAP_OK) return h->sticky;
    if (h->profiling) return QAP_ERR_INVALID_ARG;
    for (const Instance& I : h->inst)
        if (I.t != 0 || I.stepped || I.hist_cap > 0) return QAP_ERR_INVALID_ARG;  // from iteration 0, not recording
    std::vector<PlanCfg> cands;
    const bool several = h->inst.size() > 1;
    // chains beyond the runtime's hardware queues less one (the handle's
    // stream takes one) would share a queue and run one after the other
    const char* hwq = std::getenv("GPU_MAX_HW_QUEUES");
    const int queues = hwq && std::atoi(hwq) > 0 ? std::atoi(hwq) : 4;
    const int max_chains = std::max(1, std::min(kMaxChains, queues - 1));
    for (int split = 0; split <= (several ? 2 : 0); ++split)
        for (int chains = 1; chains <= max_chains; ++chains)
            for (int ipg : {0, 1, kItersPerGraph}) {
                PlanCfg c;
                c.chains = chains;
                c.split = split;
                c.ipg = ipg;
                cands.push_back(c);
            }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return QAP_ERR_DEVICE;
    }
    // every plan is timed on the same iterations: from iteration 0, the first
    // kTuneWarmup untimed (graph capture, the fast first iterations)
    auto time_plan = [&](const PlanCfg& c, int iters, float* ms) {
        int r = apply_plan(h, c);
        if (r == QAP_OK) r = reset_state(h);
        if (r == QAP_OK) r = impl_step(h, kTuneWarmup);
        hipError_t e = r == QAP_OK ? hipEventRecord(e0, h->stream) : hipSuccess;
        if (r == QAP_OK && e == hipSuccess) r = impl_step(h, iters);
        if (r == QAP_OK && e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (r == QAP_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        *ms = 0.0f;
        if (r == QAP_OK && e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
        if (r == QAP_OK && e != hipSuccess) r = dev_err(h, e);
        *ms /= (float)iters;
        return r;
    };
    // a first pass over every candidate, then a second over the fastest few, on twice the
    // iterations, in reverse order (a plan timed first is not favoured twice)
    std::vector<std::pair<float, size_t>> first;
    int rc = QAP_OK;
    for (size_t i = 0; i < cands.size() && rc == QAP_OK; ++i) {
        float ms = 0.0f;
        rc = time_plan(cands[i], trial, &ms);
        first.emplace_back(ms, i);
    }
    PlanCfg best = h->cfg;
    float best_ms = 0.0f;
    if (rc == QAP_OK) {
        std::stable_sort(first.begin(), first.end());
        const size_t keep = std::min<size_t>(kTuneFinalists, first.size());
        for (size_t j = keep; j-- > 0 && rc == QAP_OK;) {
            float ms = 0.0f;
            rc = time_plan(cands[first[j].second], 2 * trial, &ms);
            if (rc == QAP_OK && (best_ms == 0.0f || ms < best_ms)) {
                best = cands[first[j].second];
                best_ms = ms;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == QAP_OK) rc = apply_plan(h, best);
    if (rc == QAP_OK) rc = reset_state(h);  // back to iteration 0
    if (rc != QAP_OK) return rc;
    store_plan(h, best, best_ms);
    if (chosen) {
        chosen->stream_chains = best.chains;
        chosen->split = best.split;
        chosen->iters_per_graph = best.ipg;
        chosen->ms_per_iteration = best_ms;
    }
    return QAP_OK;
}

int impl_path(qap_swarm* h, int32_t instance, int32_t* delta_path, int32_t* symmetric)
{
    Instance* I;
    int rc = get_instance(h, instance, &I);
    if (rc != QAP_OK) return rc;
    if (delta_path)
        *delta_path = I->d.path == 1 ? QAP_PATH_INT8_MFMA : I->d.path == 3 ? QAP_PATH_SPLIT_MFMA : QAP_PATH_INT32;
    if (symmetric) *symmetric = I->d.sym;
    return QAP_OK;
}


}  // namespace

extern "C" {

// Entry points: no C++ exception crosses the ABI (a failed host allocation
// is QAP_ERR_NOMEM).
int qap_swarm_init_batch(const qap_instance* insts, const qap_params* prms, int32_t count, qap_swarm** out)
{
    qap_swarm* hold = nullptr;
    try {
        return impl_init_batch(insts, prms, count, out, &hold);
    } catch (const std::bad_alloc&) {
        qap_swarm_destroy(hold);
        return QAP_ERR_NOMEM;
    } catch (...) {
        qap_swarm_destroy(hold);
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_init(const qap_instance* inst, const qap_params* prm, qap_swarm** out)
{
    return qap_swarm_init_batch(inst, prm, 1, out);
}

int qap_swarm_fail_alloc(int32_t nth)
{
    if (nth < 0) return QAP_ERR_INVALID_ARG;
    g_fail_countdown.store(nth);
    return QAP_OK;
}

int64_t qap_swarm_live_allocations(void) { return g_live_allocs.load(); }

int qap_swarm_step(qap_swarm* h, int32_t iterations)
{
    try {
        return impl_step(h, iterations);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_sync(qap_swarm* h)
{
    try {
        return impl_sync(h);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_best(qap_swarm* h, int32_t instance, int64_t* goal, int32_t* perm, int32_t* iter_found)
{
    try {
        return impl_best(h, instance, goal, perm, iter_found);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_swarm_bests(qap_swarm* h, int32_t instance, int64_t* goals)
{
    try {
        return impl_swarm_bests(h, instance, goals);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_get_state(qap_swarm* h, int32_t instance, qap_state* st)
{
    try {
        return impl_get_state(h, instance, st);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_set_state(qap_swarm* h, int32_t instance, const qap_state* st)
{
    try {
        return impl_set_state(h, instance, st);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_eval(qap_swarm* h, int32_t instance, const int32_t* perms, int32_t count, int64_t* goals,
                   int64_t* deltas)
{
    try {
        return impl_eval(h, instance, perms, count, goals, deltas);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_deltas(qap_swarm* h, int32_t instance, int32_t particle, int64_t* out, int32_t* perm)
{
    try {
        return impl_deltas(h, instance, particle, out, perm);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_profile(qap_swarm* h, int32_t enable, double* stage_ms, int64_t* launches)
{
    try {
        return impl_profile(h, enable, stage_ms, launches);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_stats(qap_swarm* h, int32_t instance, int32_t nq, const int32_t* q_ppm, int64_t* swarm_q,
                    int64_t* pop_q, int32_t bins, int64_t lo, int64_t hi, int64_t* swarm_hist, int64_t* pop_hist)
{
    try {
        return impl_stats(h, instance, nq, q_ppm, swarm_q, pop_q, bins, lo, hi, swarm_hist, pop_hist);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_stats_noalloc(qap_swarm* h, int32_t instance, int32_t nq, const int32_t* q_ppm, int64_t* swarm_q,
                            int64_t* pop_q, int32_t bins, int64_t lo, int64_t hi, int64_t* swarm_hist,
                            int64_t* pop_hist)
{
    try {
        return impl_stats_noalloc(h, instance, nq, q_ppm, swarm_q, pop_q, bins, lo, hi, swarm_hist, pop_hist);
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_graph(qap_swarm* h, int32_t* active, int32_t* streams)
{
    try {
        return impl_graph(h, active, streams);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_history_start(qap_swarm* h, int32_t instance, int32_t capacity, int32_t nq, const int32_t* q_ppm,
                            int32_t bins, int64_t lo, int64_t hi)
{
    try {
        return impl_history_start(h, instance, capacity, nq, q_ppm, bins, lo, hi);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_history_stop(qap_swarm* h, int32_t instance)
{
    try {
        return impl_history_stop(h, instance);
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_history_read(qap_swarm* h, int32_t instance, int32_t max_records, int32_t* count, int32_t* iters,
                           int64_t* swarm_q, int64_t* pop_q, int64_t* swarm_hist, int64_t* pop_hist)
{
    try {
        return impl_history_read(h, instance, max_records, count, iters, swarm_q, pop_q, swarm_hist, pop_hist);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_get_plan(qap_swarm* h, qap_plan* plan)
{
    try {
        return impl_get_plan(h, plan);
    } catch (...) {
        return QAP_ERR_NOMEM;
    }
}

int qap_swarm_set_plan(qap_swarm* h, const qap_plan* plan)
{
    try {
        return impl_set_plan(h, plan);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_tune(qap_swarm* h, int32_t trial_iterations, qap_plan* chosen)
{
    try {
        return impl_tune(h, trial_iterations, chosen);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

int qap_swarm_path(qap_swarm* h, int32_t instance, int32_t* delta_path, int32_t* symmetric)
{
    try {
        return impl_path(h, instance, delta_path, symmetric);
    } catch (const std::bad_alloc&) {
        return QAP_ERR_NOMEM;
    } catch (...) {
        return QAP_ERR_DEVICE;
    }
}

}  // extern "C"
