// Batched parameter sweeps of uneven grids, kernel plans and the autotuner.
//
// A batch holds n instances (grid + pulse).  Instances of the same grid shape
// form a group whose states and spectra sit in one allocation, slot after
// slot; every pass kernel of a step runs over all active slots of a group at
// once (grid y = slot).  Slots are ordered by step count, longest first, so
// the active set of step k is a prefix.  Groups run on their own streams,
// forked from and joined back to the batch stream, and the whole run (init,
// every step of every group, every cut-out) is captured once into a hipGraph
// and replayed while the step counts, time steps, window and destination are
// unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "engine.h"

namespace {
using namespace tf::host;

// ---------------------------------------------------------------- plans
struct PlanKey {
    std::string arch;
    int prec, nx, ny, nz;
    bool operator<(const PlanKey& o) const {
        return std::tie(arch, prec, nx, ny, nz) < std::tie(o.arch, o.prec, o.nx, o.ny, o.nz);
    }
};

std::mutex g_plan_mu;
std::string g_plan_path;
bool g_plan_loaded = false;
std::map<PlanKey, KernelPlan> g_plans;

std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Plan file: '#' comments; entries
// "arch prec nx ny nz row_block fast zvariant ystrip ms" (lines without the
// ystrip field keep 64-column y strips).  False for comments and bad lines.
bool parse_plan_line(const std::string& line, PlanKey& k, KernelPlan& p, double& ms) {
    if (line.empty() || line[0] == '#') return false;
    std::istringstream is(line);
    std::vector<std::string> t;
    for (std::string w; is >> w;) t.push_back(w);
    if (t.size() != 9 && t.size() != 10) return false;
    try {
        k.arch = t[0];
        k.prec = t[1] == "f64" ? TF_F64 : TF_F32;
        k.nx = std::stoi(t[2]);
        k.ny = std::stoi(t[3]);
        k.nz = std::stoi(t[4]);
        p.row_block = std::stoi(t[5]);
        p.fast = std::stoi(t[6]) != 0;
        p.zvariant = std::stoi(t[7]);
        p.ystrip = t.size() == 10 ? std::stoi(t[8]) : 64;
        ms = std::stod(t.back());
    } catch (...) {
        return false;
    }
    return p.row_block > 0 && (p.ystrip == 64 || p.ystrip == 32);
}

void load_plans_locked() {
    if (g_plan_loaded) return;
    g_plan_loaded = true;
    g_plans.clear();
    if (g_plan_path.empty()) return;
    std::ifstream f(g_plan_path);
    std::string line;
    while (std::getline(f, line)) {
        PlanKey k;
        KernelPlan p;
        double ms = 0.0;
        if (parse_plan_line(line, k, p, ms)) g_plans[k] = p;
    }
}

void env_overrides(const tf_grid& g, KernelPlan& p) {
    if (const char* v = std::getenv("TFOCUS_ROW_BLOCK")) {
        const int b = std::atoi(v);
        if (tf::row_block_ok(b, g.ny)) p.row_block = b;
    }
    if (const char* v = std::getenv("TFOCUS_GENERIC_KERNELS")) p.fast = !(v[0] == '1');
    if (const char* v = std::getenv("TFOCUS_ZVARIANT")) p.zvariant = std::atoi(v);
    if (const char* v = std::getenv("TFOCUS_YSTRIP")) {
        const int w = std::atoi(v);
        if (w == 64 || w == 32) p.ystrip = w;
    }
}

}  // namespace

tf::host::KernelPlan tf::host::plan_for(const tf_grid& g, int precision) {
    KernelPlan p;
    p.row_block = (g.ny % 8 == 0) ? 8 : g.ny;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        if (g_plan_path.empty()) {
            if (const char* e = std::getenv("TFOCUS_PLAN_FILE")) {
                g_plan_path = e;
                g_plan_loaded = false;
            }
        }
        if (!g_plan_path.empty()) {
            load_plans_locked();
            const PlanKey k{device_arch(), precision, g.nx, g.ny, g.nz};
            auto it = g_plans.find(k);
            if (it != g_plans.end() && tf::row_block_ok(it->second.row_block, g.ny)) p = it->second;
        }
    }
    env_overrides(g, p);
    // a plan (file line or environment) whose strip offsets would not fit
    // 32 bits runs the generic kernels, which address with 64 bits
    if (p.fast && !fast_offsets_fit(g, p.row_block, precision)) p.fast = false;
    return p;
}

// ---------------------------------------------------------------- batch
namespace {

struct Group {
    tf_grid grid{};
    std::vector<int> members;        // instance ids
    std::vector<int> slot_of;        // slot -> instance id (for the current run)
    long cells = 0;
    size_t state_elems = 0, spec_elems = 0;   // per slot
    void* state = nullptr;
    void* spec = nullptr;
    void* tw[3] = {nullptr, nullptr, nullptr};
    double* cdt = nullptr;           // per slot
    tf::RowMap rm{};
    KernelPlan kp;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
};

}  // namespace

struct tf_batch {
    int prec = TF_F32;
    size_t esize = 4;
    hipStream_t stream = nullptr;
    int n = 0;
    std::vector<tf_grid> grids;
    std::vector<tf_pulse> pulses;
    std::vector<tf_pulse_info> infos;
    std::vector<int> group_of, slot_in_group;
    std::vector<Group> groups;
    std::vector<void*> tabs;               // per instance spectral table (or null)
    std::vector<tf::PulseDev> pdev;
    hipEvent_t fork = nullptr;
    hipStream_t cap = nullptr;             // private stream the sweep is captured on
    // graph cache
    hipGraphExec_t exec = nullptr;
    std::vector<int64_t> key_steps;
    std::vector<double> key_dt;
    tf_window key_win{};
    void* key_dst = nullptr;
};

namespace {

void batch_free(tf_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    for (Group& g : b->groups) {
        void* ps[] = {g.state, g.spec, g.tw[0], g.tw[1], g.tw[2], g.cdt};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        if (g.stream) (void)hipStreamDestroy(g.stream);
        if (g.done) (void)hipEventDestroy(g.done);
    }
    for (void* t : b->tabs)
        if (t) (void)hipFree(t);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->cap) (void)hipStreamDestroy(b->cap);
}

bool same_grid(const tf_grid& a, const tf_grid& b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.dx == b.dx && a.dy == b.dy && a.dz == b.dz &&
           a.x_min == b.x_min && a.y_min == b.y_min && a.z_min == b.z_min && a.replicate_yz == b.replicate_yz;
}

// Window node indices of instance i (host); false if outside the grid.
bool window_origin(const tf_grid& g, const tf_window& w, long& ic, long& jc, long& kc) {
    ic = (long)std::floor((w.cx - g.x_min) / g.dx + 0.5);
    jc = (long)std::floor((w.cy - g.y_min) / g.dy + 0.5);
    kc = (long)std::floor((w.cz - g.z_min) / g.dz + 0.5);
    const long j0 = jc - w.wy / 2, k0 = kc - w.wz / 2;
    return g.replicate_yz || (j0 >= 0 && j0 + w.wy <= g.ny && k0 >= 0 && k0 + w.wz <= g.nz);
}

template <typename T>
hipError_t enqueue_group(tf_batch* b, Group& G, const int64_t* nsteps, const double* dt, const tf_window& w,
                         void* dst) {
    const size_t wsize = 6 * (size_t)w.wx * w.wy * w.wz;
    const tf::GridDev gd = grid_dev(G.grid);
    const int nslot = (int)G.slot_of.size();
    hipError_t e = hipSuccess;
    for (int s = 0; s < nslot && e == hipSuccess; ++s) {
        const int i = G.slot_of[s];
        e = tf::launch_init_map<T>(static_cast<T*>(G.state) + s * G.state_elems, gd, b->pdev[i], G.stream);
    }
    const int64_t kmax = nslot ? nsteps[G.slot_of[0]] : 0;
    for (int64_t k = 0; k < kmax && e == hipSuccess; ++k) {
        int active = 0;
        while (active < nslot && nsteps[G.slot_of[active]] > k) ++active;
        tf::Batch bt;
        bt.n = active;
        bt.sreal = (long)G.state_elems;
        bt.sspec = (long)(G.spec_elems / 2);
        bt.cdt = G.cdt;
        e = step_passes<T>(G.state, G.spec, G.tw, G.grid, G.rm, G.kp, 0.0, k == 0, bt, G.stream);
    }
    for (int s = 0; s < nslot && e == hipSuccess; ++s) {
        const int i = G.slot_of[s];
        long ic, jc, kc;
        window_origin(G.grid, w, ic, jc, kc);
        const double t = 0.0 + (double)nsteps[i] * dt[i];
        e = tf::launch_readout<T>(static_cast<const T*>(G.state) + s * G.state_elems,
                                  static_cast<T*>(dst) + i * wsize, gd, w.wx, w.wy, w.wz, ic, jc, kc, t,
                                  b->infos[i].R_min, b->infos[i].R_max, G.stream);
    }
    return e;
}

// Enqueue a whole sweep behind `origin`: fork to the group streams, join back.
hipError_t enqueue_run(tf_batch* b, hipStream_t origin, const int64_t* nsteps, const double* dt, const tf_window& w,
                       void* dst) {
    hipError_t e = hipEventRecord(b->fork, origin);
    for (Group& G : b->groups) {
        if (e != hipSuccess) break;
        e = hipStreamWaitEvent(G.stream, b->fork, 0);
        if (e != hipSuccess) break;
        e = b->prec == TF_F64 ? enqueue_group<double>(b, G, nsteps, dt, w, dst)
                              : enqueue_group<float>(b, G, nsteps, dt, w, dst);
        if (e != hipSuccess) break;
        e = hipEventRecord(G.done, G.stream);
        if (e != hipSuccess) break;
        e = hipStreamWaitEvent(origin, G.done, 0);
    }
    return e;
}

// Tuning state (tf_tune): a hash of the element index mapped to [-1, 1), so that the
// timed passes move ordinary nonzero data (grid-stride over n elements).
template <typename T>
__global__ void k_tune_fill(T* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        p[i] = T((double)(h >> 8) * (1.0 / 8388608.0) - 1.0);
    }
}

// Device buffers and events of one tuning size, released on every return
// path (the device is synchronised first, so no queued work still uses them).
struct TuneBuffers {
    void* state = nullptr;
    void* spec = nullptr;
    void* tw[3] = {nullptr, nullptr, nullptr};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TuneBuffers() = default;
    TuneBuffers(const TuneBuffers&) = delete;
    TuneBuffers& operator=(const TuneBuffers&) = delete;
    ~TuneBuffers() {
        (void)hipDeviceSynchronize();
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (void* p : {state, spec, tw[0], tw[1], tw[2]})
            if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" {

tf_status tf_batch_create(const tf_grid* grids, const tf_pulse* pulses, int32_t n, int32_t precision,
                          void* hip_stream, tf_batch** out) {
    if (!grids || !pulses || !out || n <= 0) return fail(TF_EINVAL, "grids, pulses, out must be non-NULL and n > 0");
    *out = nullptr;
    if (precision != TF_F32 && precision != TF_F64) return fail(TF_EINVAL, "precision must be TF_F32 or TF_F64");
    tf_batch* b = new tf_batch();
    b->prec = precision;
    b->esize = precision == TF_F64 ? 8 : 4;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->n = n;
    b->grids.assign(grids, grids + n);
    b->pulses.assign(pulses, pulses + n);
    b->infos.resize(n);
    b->group_of.resize(n);
    b->tabs.assign(n, nullptr);
    b->pdev.resize(n);
    size_t need = 0;
    for (int i = 0; i < n; ++i) {
        tf_status st = validate_grid(&grids[i]);
        if (st == TF_OK) st = validate_pulse(&pulses[i]);
        if (st != TF_OK) {
            delete b;
            return fail(st, "instance " + std::to_string(i) + ": " + last_error());
        }
        geometry(&pulses[i], &b->infos[i]);
        b->infos[i].D = grids[i].nx * grids[i].dx;
        b->infos[i].overlap = b->infos[i].D < b->infos[i].D_min ? 1 : 0;
        if (!(b->infos[i].D > pulses[i].L)) {
            delete b;
            return fail(TF_EDOMAIN, "instance " + std::to_string(i) + ": layer period must exceed L");
        }
        int gi = -1;
        for (size_t k = 0; k < b->groups.size(); ++k)
            if (same_grid(b->groups[k].grid, grids[i])) gi = (int)k;
        if (gi < 0) {
            b->groups.emplace_back();
            b->groups.back().grid = grids[i];
            gi = (int)b->groups.size() - 1;
        }
        b->groups[gi].members.push_back(i);
        b->group_of[i] = gi;
        const size_t cells = (size_t)grids[i].nx * grids[i].ny * grids[i].nz;
        need += 12 * cells * b->esize;
    }
    if (need > device_cap()) {
        delete b;
        return fail(TF_ENOMEM, "batch needs " + std::to_string(need) + " device bytes, above TFOCUS_MAX_DEVICE_BYTES");
    }
    auto alloc = [&](void** p, size_t bytes) -> tf_status {
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipErrorOutOfMemory) return fail(TF_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        if (e != hipSuccess) return fail(TF_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
        return TF_OK;
    };
    tf_status st = TF_OK;
    for (Group& G : b->groups) {
        if (st != TF_OK) break;
        const tf_grid& g = G.grid;
        G.cells = (long)g.nx * g.ny * g.nz;
        G.state_elems = 6 * (size_t)G.cells;
        G.spec_elems = 2 * 6 * (size_t)g.nz * g.ny * tf::nkx_of(g.nx);
        G.kp = plan_for(g, precision);
        G.rm = tf::RowMap(g.ny, g.nz, G.kp.row_block);
        const size_t m = G.members.size();
        st = alloc(&G.state, m * G.state_elems * b->esize);
        if (st == TF_OK) st = alloc(&G.spec, m * G.spec_elems * b->esize);
        const int ns[3] = {g.nx, g.ny, g.nz};
        for (int a = 0; a < 3 && st == TF_OK; ++a) st = alloc(&G.tw[a], 2 * b->esize * ns[a]);
        if (st == TF_OK) st = alloc((void**)&G.cdt, m * sizeof(double));
        if (st == TF_OK && hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking) != hipSuccess)
            st = fail(TF_EDEVICE, "hipStreamCreate failed");
        if (st == TF_OK && hipEventCreateWithFlags(&G.done, hipEventDisableTiming) != hipSuccess)
            st = fail(TF_EDEVICE, "hipEventCreate failed");
        for (int a = 0; a < 3 && st == TF_OK; ++a)
            if (upload_twiddles(G.tw[a], ns[a], precision, b->stream) != hipSuccess)
                st = fail(TF_EDEVICE, "twiddle upload failed");
    }
    if (st == TF_OK && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        st = fail(TF_EDEVICE, "hipEventCreate failed");
    if (st == TF_OK && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        st = fail(TF_EDEVICE, "hipStreamCreate failed");
    for (int i = 0; i < n && st == TF_OK; ++i) {
        b->pdev[i] = pulse_dev(&pulses[i], b->infos[i]);
        std::vector<double> all;
        size_t spec_len = 0;
        double gnorm = 1.0;
        int nfreq = 0;
        st = pulse_tables(&pulses[i], all, spec_len, gnorm, nfreq);
        if (st != TF_OK) {
            st = fail(st, "instance " + std::to_string(i) + ": " + last_error());
            break;
        }
        if (!all.empty()) {
            st = alloc(&b->tabs[i], all.size() * sizeof(double));
            if (st == TF_OK &&
                hipMemcpy(b->tabs[i], all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                st = fail(TF_EDEVICE, "pulse table upload failed");
            if (st == TF_OK)
                pulse_dev_tables(b->pdev[i], &pulses[i], static_cast<const double*>(b->tabs[i]), spec_len, gnorm,
                                 nfreq);
        }
    }
    if (st != TF_OK) {
        batch_free(b);
        delete b;
        return st;
    }
    *out = b;
    return TF_OK;
}

tf_status tf_batch_run(tf_batch* b, const int64_t* nsteps, const double* dt, const tf_window* w, void* dst_dev,
                       int32_t use_graph) {
    if (!b || !nsteps || !dt || !w || !dst_dev) return fail(TF_EINVAL, "batch, nsteps, dt, window, dst must be non-NULL");
    if (w->wx <= 0 || w->wy <= 0 || w->wz <= 0) return fail(TF_EINVAL, "window sizes must be > 0");
    for (int i = 0; i < b->n; ++i) {
        if (nsteps[i] < 0) return fail(TF_EINVAL, "nsteps must be >= 0");
        if (!std::isfinite(dt[i])) return fail(TF_EINVAL, "dt must be finite");
        long ic, jc, kc;
        if (!window_origin(b->grids[i], *w, ic, jc, kc))
            return fail(TF_EINVAL, "window leaves the transverse extent of instance " + std::to_string(i));
    }
    const bool cached = b->exec && use_graph && b->key_dst == dst_dev &&
                        std::equal(nsteps, nsteps + b->n, b->key_steps.begin()) &&
                        std::equal(dt, dt + b->n, b->key_dt.begin()) && !std::memcmp(&b->key_win, w, sizeof(*w));
    if (!cached) {
        // the slot order and the per-slot dt below are what a captured graph
        // reads: once they are rewritten, no earlier graph may be replayed
        if (b->exec) {
            TF_HIP(hipStreamSynchronize(b->stream));
            TF_HIP(hipGraphExecDestroy(b->exec));
            b->exec = nullptr;
        }
        b->key_steps.clear();
        b->key_dt.clear();
        b->key_dst = nullptr;
        // slot order: longest run first, so the active slots of a step are a prefix
        for (Group& G : b->groups) {
            G.slot_of = G.members;
            std::stable_sort(G.slot_of.begin(), G.slot_of.end(),
                             [&](int a, int c) { return nsteps[a] > nsteps[c]; });
            std::vector<double> c(G.slot_of.size());
            for (size_t s = 0; s < c.size(); ++s) c[s] = dt[G.slot_of[s]];
            TF_HIP(hipMemcpyAsync(G.cdt, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, b->stream));
        }
        TF_HIP(hipStreamSynchronize(b->stream));
    }
    if (!use_graph) {
        hipError_t e = enqueue_run(b, b->stream, nsteps, dt, *w, dst_dev);
        if (e != hipSuccess) return fail(TF_EDEVICE, std::string("batch run: ") + hipGetErrorString(e));
        return TF_OK;
    }
    if (!cached) {
        hipGraph_t graph = nullptr;
        TF_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_run(b, b->cap, nsteps, dt, *w, dst_dev);
        hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(TF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return fail(TF_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        b->key_steps.assign(nsteps, nsteps + b->n);
        b->key_dt.assign(dt, dt + b->n);
        b->key_win = *w;
        b->key_dst = dst_dev;
    }
    TF_HIP(hipGraphLaunch(b->exec, b->stream));
    return TF_OK;
}

tf_status tf_batch_get_fields(tf_batch* b, int32_t i, void* dst, int32_t dst_on_device) {
    if (!b || !dst || i < 0 || i >= b->n) return fail(TF_EINVAL, "bad batch, index or dst");
    const Group& G = b->groups[b->group_of[i]];
    int slot = -1;
    for (size_t s = 0; s < G.slot_of.size(); ++s)
        if (G.slot_of[s] == i) slot = (int)s;
    if (slot < 0) return fail(TF_ESTATE, "instance has not been run");
    const size_t bytes = G.state_elems * b->esize;
    const char* src = static_cast<const char*>(G.state) + slot * bytes;
    TF_HIP(hipMemcpyAsync(dst, src, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream));
    if (!dst_on_device) TF_HIP(hipStreamSynchronize(b->stream));
    return TF_OK;
}

tf_status tf_batch_destroy(tf_batch* b) {
    if (!b) return TF_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    for (Group& G : b->groups)
        if (G.stream) (void)hipStreamSynchronize(G.stream);
    batch_free(b);
    delete b;
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("tf_batch_destroy: ") + hipGetErrorString(e));
    return TF_OK;
}

tf_status tf_kernel_plan(const tf_grid* grid, int32_t precision, int32_t* row_block, int32_t* fast,
                         int32_t* zvariant, int32_t* ystrip) {
    if (precision != TF_F32 && precision != TF_F64) return fail(TF_EINVAL, "precision must be TF_F32 or TF_F64");
    tf_status st = validate_grid(grid);
    if (st != TF_OK) return st;
    const KernelPlan p = plan_for(*grid, precision);
    if (row_block) *row_block = p.row_block;
    if (fast) *fast = p.fast ? 1 : 0;
    if (zvariant) *zvariant = p.zvariant;
    if (ystrip) *ystrip = p.ystrip;
    return TF_OK;
}

tf_status tf_set_plan_file(const char* path) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plan_path = path ? path : "";
    g_plan_loaded = false;
    return TF_OK;
}

// Autotuner: for every cube size, time a few steps of each kernel plan on a
// pseudo-random state with HIP events, in three interleaved rounds, and keep
// the fastest; results are merged into the plan file (entries of other
// sizes/precisions/architectures are kept).
tf_status tf_tune(const int32_t* sizes, int32_t n, int32_t precision, const char* plan_path, double* best_ms) {
    if (!sizes || n <= 0 || !plan_path) return fail(TF_EINVAL, "sizes, n > 0 and plan_path required");
    if (precision != TF_F32 && precision != TF_F64) return fail(TF_EINVAL, "precision must be TF_F32 or TF_F64");
    for (int i = 0; i < n; ++i)
        if (!length_ok(sizes[i]) || sizes[i] % 2) return fail(TF_EUNSUPPORTED, "size " + std::to_string(sizes[i]));
    const std::string arch = device_arch();
    const size_t es = precision == TF_F64 ? 8 : 4;
    std::map<PlanKey, std::pair<KernelPlan, double>> found;
    for (int i = 0; i < n; ++i) {
        const int N = sizes[i];
        tf_grid g{};
        g.nx = g.ny = g.nz = N;
        g.dx = g.dy = g.dz = 1.0;
        const size_t cells = (size_t)N * N * N;
        TuneBuffers tb;
        TF_HIP(hipMalloc(&tb.state, 6 * cells * es));
        TF_HIP(hipMalloc(&tb.spec, 6 * cells * es));
        for (int a = 0; a < 3; ++a) {
            TF_HIP(hipMalloc(&tb.tw[a], 2 * es * N));
            TF_HIP(upload_twiddles(tb.tw[a], N, precision, nullptr));
        }
        if (precision == TF_F64) hipLaunchKernelGGL(k_tune_fill<double>, dim3(1024), dim3(256), 0, nullptr, (double*)tb.state, 6 * cells);
        else hipLaunchKernelGGL(k_tune_fill<float>, dim3(1024), dim3(256), 0, nullptr, (float*)tb.state, 6 * cells);
        TF_HIP(hipGetLastError());
        std::vector<KernelPlan> cands;
        for (int rb : {8, N}) {
            KernelPlan p;
            p.row_block = rb;
            p.fast = false;
            cands.push_back(p);
            if (!fast_offsets_fit(g, rb, precision)) continue;
            // variants 7 to 9 and 11 (one wave per mode) exist for
            // 512-point z columns, 7 and 8 for 256-point ones; elsewhere
            // they run variant 6.  Variant 10 (float32
            // phases) is left to explicit plans: its phase error is the same
            // on every step, so it grows linearly with the step count, for
            // about 1% of the z pass's time
            for (int ys : {64, 32})
                for (int zv = 0; zv < (N == 512 ? 12 : N == 256 ? 9 : 7); ++zv) {
                    if (zv == 10) continue;
                    p.fast = true;
                    p.zvariant = zv;
                    p.ystrip = ys;
                    cands.push_back(p);
                }
        }
        TF_HIP(hipEventCreate(&tb.e0));
        TF_HIP(hipEventCreate(&tb.e1));
        KernelPlan best;
        double bms = 1e300;
        const int reps = N >= 256 ? 4 : 10;
        // candidates are timed in interleaved rounds and keep their fastest
        // round, so that clock ramp-up and drift favour none of them
        constexpr int ROUNDS = 3;
        std::vector<double> tmin(cands.size(), 1e300);
        for (int round = 0; round < ROUNDS; ++round)
            for (size_t ci = 0; ci < cands.size(); ++ci) {
                const KernelPlan& p = cands[ci];
                tf::RowMap rm{N, N, p.row_block};
                hipError_t e = hipSuccess;
                for (int r = 0; r < 2 && e == hipSuccess; ++r)
                    e = precision == TF_F64
                            ? step_passes<double>(tb.state, tb.spec, tb.tw, g, rm, p, 0.1, false, tf::Batch{}, nullptr)
                            : step_passes<float>(tb.state, tb.spec, tb.tw, g, rm, p, 0.1, false, tf::Batch{}, nullptr);
                TF_HIP(hipEventRecord(tb.e0, nullptr));
                for (int r = 0; r < reps && e == hipSuccess; ++r)
                    e = precision == TF_F64
                            ? step_passes<double>(tb.state, tb.spec, tb.tw, g, rm, p, 0.1, false, tf::Batch{}, nullptr)
                            : step_passes<float>(tb.state, tb.spec, tb.tw, g, rm, p, 0.1, false, tf::Batch{}, nullptr);
                TF_HIP(hipEventRecord(tb.e1, nullptr));
                TF_HIP(hipEventSynchronize(tb.e1));
                if (e != hipSuccess) return fail(TF_EDEVICE, std::string("tuning step: ") + hipGetErrorString(e));
                float ms = 0.0f;
                TF_HIP(hipEventElapsedTime(&ms, tb.e0, tb.e1));
                tmin[ci] = std::min(tmin[ci], double(ms) / reps);
            }
        for (size_t ci = 0; ci < cands.size(); ++ci)
            if (tmin[ci] < bms) {
                bms = tmin[ci];
                best = cands[ci];
            }
        found[PlanKey{arch, precision, N, N, N}] = {best, bms};
        if (best_ms) best_ms[i] = bms;
    }
    // merge into the plan file
    std::map<PlanKey, std::pair<KernelPlan, double>> all;
    {
        std::ifstream f(plan_path);
        std::string line;
        while (std::getline(f, line)) {
            PlanKey k;
            KernelPlan p;
            double ms = 0.0;
            if (parse_plan_line(line, k, p, ms)) all[k] = {p, ms};
        }
    }
    for (auto& kv : found) all[kv.first] = kv.second;
    std::ofstream f(plan_path);
    if (!f) return fail(TF_EINVAL, std::string("cannot write ") + plan_path);
    f << "# tfocus kernel plans: arch precision nx ny nz row_block fast zvariant ystrip ms_per_step\n";
    for (auto& kv : all) {
        const PlanKey& k = kv.first;
        const KernelPlan& p = kv.second.first;
        char buf[256];
        std::snprintf(buf, sizeof(buf), "%s %s %d %d %d %d %d %d %d %.4f\n", k.arch.c_str(),
                      k.prec == TF_F64 ? "f64" : "f32", k.nx, k.ny, k.nz, p.row_block, p.fast ? 1 : 0, p.zvariant,
                      p.ystrip, kv.second.second);
        f << buf;
    }
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plan_loaded = false;
    }
    return TF_OK;
}

}  // extern "C"
