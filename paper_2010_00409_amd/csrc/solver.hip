// Host engine behind the single-grid part of the C ABI (include/tfocus.h):
// buffers, pulse initialisation, the step driver, cut-out, diagnostics and
// per-launch profiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"


namespace {
using namespace tf::host;
}  // namespace

std::string& tf::host::last_error() {
    static thread_local std::string e;
    return e;
}

struct tf_solver {
    tf_grid grid{};
    int prec = TF_F32;
    size_t esize = 4;
    hipStream_t stream = nullptr;
    long cells = 0;
    int nkx = 0;
    void* state = nullptr;
    void* spec = nullptr;
    void* tw[3] = {nullptr, nullptr, nullptr};
    double* partials = nullptr;
    size_t npartials = 0;
    double* results = nullptr;     // 8 doubles
    void* pulse_tab = nullptr;
    void* dcbuf = nullptr;         // diagnostics: packed kx = 0 slot after the forward z FFT
    tf::RowMap rm{};
    bool fast = true;              // use the specialised float32 column kernels
    int ystrip = 64;               // columns per strip of the fast y kernel
    int zvariant = 0;
    void* scratch_out = nullptr;
    size_t scratch_bytes = 0;
    // current steps (tf_advance_current): the current in components 0..2 of
    // a six-component real array (3..5 stay zero) and its half spectrum
    void* jstate = nullptr;
    void* jspec = nullptr;
    double t = 0.0;
    bool project_b_next = false;
    bool have_cutout = false;
    double R_min = 0.0, R_max = 0.0;
    // per-launch timing (tf_profile)
    bool prof = false;
    std::vector<hipEvent_t> evpool;
    std::vector<int> rec_kind;
    // GRAPH_STEPS steps of one dt, captured once on a private stream and
    // replayed on `stream` by tf_advance
    hipStream_t cap = nullptr;
    hipGraphExec_t step_exec = nullptr;
    double step_dt = 0.0;
};

namespace {

// Runs launch() and, while profiling, brackets it with a pair of events.
template <class F>
hipError_t timed(tf_solver* s, int kind, F launch) {
    if (!s->prof) return launch();
    const size_t i = s->rec_kind.size();
    while (s->evpool.size() < 2 * (i + 1)) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return e;
        s->evpool.push_back(ev);
    }
    hipError_t e = hipEventRecord(s->evpool[2 * i], s->stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(s->evpool[2 * i + 1], s->stream);
    if (e == hipSuccess) s->rec_kind.push_back(kind);
    return e;
}

template <typename T>
hipError_t forward_xy(tf_solver* s, int kind_x, int kind_y) {
    const tf_grid& g = s->grid;
    hipError_t e = timed(s, kind_x, [&] {
        return tf::launch_x_forward<T>(static_cast<const T*>(s->state), s->spec, s->tw[0], g.nx, g.ny, g.nz, s->rm,
                                       tf::Batch{}, s->stream);
    });
    if (e != hipSuccess) return e;
    return timed(s, kind_y, [&] {
        return tf::launch_y_pass<T>(s->spec, s->tw[1], g.nx, g.ny, g.nz, -1, s->rm, s->fast ? s->ystrip : 0,
                                    tf::Batch{}, s->stream);
    });
}

// One step of Eqs. (1)-(2) with the current in s->jstate: the current and
// the fields are x- and y-transformed, the z pass applies the update, and
// the fields go back as in a vacuum step.
template <typename T>
hipError_t current_step(tf_solver* s, double dt, bool project_b) {
    const tf_grid& g = s->grid;
    const int ys = s->fast ? s->ystrip : 0;
    hipError_t e = timed(s, TF_PASS_OTHER, [&] {
        return tf::launch_x_forward<T>(static_cast<const T*>(s->jstate), s->jspec, s->tw[0], g.nx, g.ny, g.nz, s->rm,
                                       tf::Batch{}, s->stream);
    });
    if (e != hipSuccess) return e;
    e = timed(s, TF_PASS_OTHER, [&] {
        return tf::launch_y_pass<T>(s->jspec, s->tw[1], g.nx, g.ny, g.nz, -1, s->rm, ys, tf::Batch{}, s->stream);
    });
    if (e != hipSuccess) return e;
    e = forward_xy<T>(s, TF_PASS_X_FORWARD, TF_PASS_Y_FORWARD);
    if (e != hipSuccess) return e;
    tf::StepParams p = step_params(s->grid, dt, project_b, s->zvariant);
    e = timed(s, TF_PASS_Z_STEP, [&] {
        return tf::launch_z_current<T>(s->spec, s->jspec, s->tw[2], p, s->rm, s->stream);
    });
    if (e != hipSuccess) return e;
    e = timed(s, TF_PASS_Y_INVERSE, [&] {
        return tf::launch_y_pass<T>(s->spec, s->tw[1], g.nx, g.ny, g.nz, +1, s->rm, ys, tf::Batch{}, s->stream);
    });
    if (e != hipSuccess) return e;
    return timed(s, TF_PASS_X_INVERSE, [&] {
        return tf::launch_x_inverse<T>(s->spec, static_cast<T*>(s->state), s->tw[0], g.nx, g.ny, g.nz, s->rm,
                                       tf::Batch{}, s->stream);
    });
}

// One step; with diag_blocks the z pass is the generic kernel that also
// writes the diagnostics of the new state into s->partials (Z_STEP_DIAG),
// and *diag_blocks receives its count of 4-wide partials.
template <typename T>
hipError_t one_step(tf_solver* s, double dt, bool project_b, int* diag_blocks = nullptr) {
    const tf_grid& g = s->grid;
    hipError_t e = forward_xy<T>(s, TF_PASS_X_FORWARD, TF_PASS_Y_FORWARD);
    if (e != hipSuccess) return e;
    tf::StepParams p = step_params(s->grid, dt, project_b, s->zvariant);
    e = timed(s, TF_PASS_Z_STEP, [&] {
        if (diag_blocks)
            return tf::launch_z_pass<T>(s->spec, s->tw[2], p, s->rm, tf::Z_STEP_DIAG, s->partials, s->dcbuf,
                                        diag_blocks, false, tf::Batch{}, s->stream);
        return tf::launch_z_pass<T>(s->spec, s->tw[2], p, s->rm, tf::Z_STEP, nullptr, nullptr, nullptr, s->fast,
                                    tf::Batch{}, s->stream);
    });
    if (e != hipSuccess) return e;
    e = timed(s, TF_PASS_Y_INVERSE, [&] {
        return tf::launch_y_pass<T>(s->spec, s->tw[1], g.nx, g.ny, g.nz, +1, s->rm, s->fast ? s->ystrip : 0,
                                    tf::Batch{}, s->stream);
    });
    if (e != hipSuccess) return e;
    return timed(s, TF_PASS_X_INVERSE, [&] {
        return tf::launch_x_inverse<T>(s->spec, static_cast<T*>(s->state), s->tw[0], g.nx, g.ny, g.nz, s->rm,
                                       tf::Batch{}, s->stream);
    });
}

// Steps per captured graph: the launch cost of the remaining steps is one
// graph launch per GRAPH_STEPS steps.
constexpr int64_t GRAPH_STEPS = 8;

// The graph of GRAPH_STEPS steps of dt (without the B projection), captured
// on first use and again whenever dt changes.
template <typename T>
tf_status step_graph(tf_solver* s, double dt) {
    if (s->step_exec && std::memcmp(&s->step_dt, &dt, sizeof dt) == 0) return TF_OK;
    if (!s->cap) TF_HIP(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
    if (s->step_exec) {
        TF_HIP(hipGraphExecDestroy(s->step_exec));
        s->step_exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    TF_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
    hipStream_t user = s->stream;
    s->stream = s->cap;                       // the pass launchers enqueue on s->stream
    hipError_t e = hipSuccess;
    for (int64_t k = 0; k < GRAPH_STEPS && e == hipSuccess; ++k) e = one_step<T>(s, dt, false);
    s->stream = user;
    hipError_t e2 = hipStreamEndCapture(s->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(TF_EDEVICE, std::string("step graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&s->step_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        s->step_exec = nullptr;
        return fail(TF_EDEVICE, std::string("step graph instantiate: ") + hipGetErrorString(e));
    }
    s->step_dt = dt;
    return TF_OK;
}

void free_all(tf_solver* s) {
    if (s->step_exec) (void)hipGraphExecDestroy(s->step_exec);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    s->step_exec = nullptr;
    s->cap = nullptr;
    for (hipEvent_t ev : s->evpool) (void)hipEventDestroy(ev);
    s->evpool.clear();
    void* ptrs[] = {s->state, s->spec, s->tw[0], s->tw[1], s->tw[2], s->partials, s->results,
                    s->pulse_tab, s->dcbuf, s->scratch_out, s->jstate, s->jspec};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

// ---- allocation-free stepping (tf_advance_noalloc) ----

// Device scratch of tf_advance_noalloc: the twiddle tables of the three axes,
// then the half spectrum of the grid being advanced.  One copy per device,
// held until the process ends; every call on a device reuses it.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of this device's scratch array, looked up once per device
// with that device current.  The array's name is only a host-side stand-in.
tf_status noalloc_scratch(int dev, void** out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(TF_EUNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        TF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(TF_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TF_OK;
}

// Bytes of scratch tf_advance_noalloc needs for a grid: the twiddle tables
// (nx + ny + nz complex, rounded up to 256 bytes), then the half spectrum.
size_t noalloc_tw_bytes(const tf_grid& g, size_t esize) {
    return (2 * esize * (size_t)(g.nx + g.ny + g.nz) + 255) / 256 * 256;
}
size_t noalloc_spec_bytes(const tf_grid& g, size_t esize) {
    return (size_t)g.nz * g.ny * tf::nkx_of(g.nx) * 6 * 2 * esize;
}

// Twiddle tables of the three axes, exp(-2 pi i e / n) for e < n, laid out
// x, then y, then z (interleaved re, im): the float64 angle 2 pi e / n and its
// sine and cosine, rounded to the element type.
template <typename T>
__global__ void k_noalloc_twiddles(T* tw, int nx, int ny, int nz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx + ny + nz) return;
    int n = nx, e = i;
    if (i >= nx + ny) { n = nz; e = i - nx - ny; }
    else if (i >= nx) { n = ny; e = i - nx; }
    const double a = 2.0 * M_PI * (double)e / (double)n;
    double sn, cs;
    sincos(a, &sn, &cs);
    tw[2 * i] = T(cs);
    tw[2 * i + 1] = T(-sn);
}

template <typename T>
hipError_t noalloc_steps(const tf_grid& g, void* state, unsigned char* base, int64_t nsteps, double dt,
                         bool project_b_first, int precision, hipStream_t st) {
    const size_t es = sizeof(T);
    T* tw = reinterpret_cast<T*>(base);
    void* spec = base + noalloc_tw_bytes(g, es);
    const int nt = g.nx + g.ny + g.nz;
    hipLaunchKernelGGL(k_noalloc_twiddles<T>, dim3((nt + 255) / 256), dim3(256), 0, st, tw, g.nx, g.ny, g.nz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* tws[3] = {tw, tw + 2 * g.nx, tw + 2 * (g.nx + g.ny)};
    const KernelPlan kp = plan_for(g, precision);
    const tf::RowMap rm{g.ny, g.nz, kp.row_block};
    for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k)
        e = step_passes<T>(state, spec, tws, g, rm, kp, dt, project_b_first && k == 0, tf::Batch{}, st);
    return e;
}

}  // namespace

extern "C" {

tf_status tf_advance_noalloc(const tf_grid* grid, int32_t precision, void* state_dev, int64_t nsteps, double dt,
                             int32_t project_b_first, void* hip_stream) {
    if (!state_dev) return fail(TF_EINVAL, "state_dev is NULL");
    if (precision != TF_F32 && precision != TF_F64) return fail(TF_EINVAL, "precision must be TF_F32 or TF_F64");
    tf_status vs = validate_grid(grid);
    if (vs != TF_OK) return vs;
    if (nsteps < 0) return fail(TF_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt)) return fail(TF_EINVAL, "dt must be finite");
    const size_t es = precision == TF_F64 ? 8 : 4;
    const size_t need = noalloc_tw_bytes(*grid, es) + noalloc_spec_bytes(*grid, es);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(TF_ENOMEM, "grid needs " + std::to_string(need) + " bytes of scratch; the allocation-free path holds " +
                                   std::to_string(NOALLOC_SCRATCH_BYTES));
    int dev = 0;
    TF_HIP(hipGetDevice(&dev));
    void* base = nullptr;
    tf_status st = noalloc_scratch(dev, &base);
    if (st != TF_OK) return st;
    if (nsteps == 0) return TF_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const hipError_t e =
        precision == TF_F64
            ? noalloc_steps<double>(*grid, state_dev, static_cast<unsigned char*>(base), nsteps, dt, project_b_first != 0,
                                    precision, stream)
            : noalloc_steps<float>(*grid, state_dev, static_cast<unsigned char*>(base), nsteps, dt, project_b_first != 0,
                                   precision, stream);
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("tf_advance_noalloc: ") + hipGetErrorString(e));
    return TF_OK;
}

const char* tf_version(void) { return "tfocus 0.1"; }

const char* tf_last_error(void) { return last_error().c_str(); }

int32_t tf_supported_length(int32_t n) { return length_ok(n) ? 1 : 0; }

tf_status tf_pulse_geometry(const tf_pulse* pulse, tf_pulse_info* info) {
    if (!info) return fail(TF_EINVAL, "info is NULL");
    tf_status st = validate_pulse(pulse);
    if (st != TF_OK) return st;
    geometry(pulse, info);
    return TF_OK;
}

tf_status tf_layer_grid(const tf_pulse* pulse, int32_t nx, int32_t ny, int32_t nz, double dx, double dy,
                        double dz, tf_grid* out) {
    if (!out) return fail(TF_EINVAL, "out is NULL");
    tf_status st = validate_pulse(pulse);
    if (st != TF_OK) return st;
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(TF_EINVAL, "grid sizes must be > 0");
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz)) return fail(TF_EINVAL, "spacings must be > 0");
    tf_pulse_info g;
    geometry(pulse, &g);
    const double D = nx * dx;
    const double i0 = std::floor((g.R_min + D) / dx + 0.5);
    std::memset(out, 0, sizeof(*out));
    out->nx = nx; out->ny = ny; out->nz = nz;
    out->dx = dx; out->dy = dy; out->dz = dz;
    out->x_min = -i0 * dx;
    out->y_min = -(double)(ny / 2) * dy;
    out->z_min = -(double)(nz / 2) * dz;
    return TF_OK;
}

tf_status tf_create(const tf_grid* grid, int32_t precision, void* hip_stream, tf_solver** out) {
    if (!grid || !out) return fail(TF_EINVAL, "grid and out must not be NULL");
    *out = nullptr;
    if (precision != TF_F32 && precision != TF_F64) return fail(TF_EINVAL, "precision must be TF_F32 or TF_F64");
    {
        tf_status vs = validate_grid(grid);
        if (vs != TF_OK) return vs;
    }
    tf_solver* s = new tf_solver();
    s->grid = *grid;
    s->prec = precision;
    s->esize = precision == TF_F64 ? 8 : 4;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->cells = (long)grid->nx * grid->ny * grid->nz;
    s->nkx = tf::nkx_of(grid->nx);
    const size_t state_b = 6 * (size_t)s->cells * s->esize;
    const size_t spec_b = (size_t)grid->nz * grid->ny * s->nkx * 6 * 2 * s->esize;
    const int zb = precision == TF_F64 ? tf::z_diag_blocks<double>(grid->nx, grid->ny, grid->nz)
                                       : tf::z_diag_blocks<float>(grid->nx, grid->ny, grid->nz);
    s->npartials = std::max<size_t>(tf::SUMSQ_BLOCKS, (size_t)zb * 5);
    const size_t tw_b = 2 * s->esize * (size_t)(grid->nx + grid->ny + grid->nz);
    const size_t dc_b = (size_t)grid->ny * grid->nz * 6 * 2 * s->esize;
    const size_t need = state_b + spec_b + tw_b + dc_b + s->npartials * 8 + 64;
    const KernelPlan kp = plan_for(*grid, precision);
    s->rm = tf::RowMap(grid->ny, grid->nz, kp.row_block);
    s->fast = kp.fast;
    s->zvariant = kp.zvariant;
    s->ystrip = kp.ystrip;
    if (need > device_cap()) {
        delete s;
        return fail(TF_ENOMEM, "solver needs " + std::to_string(need) + " device bytes, above TFOCUS_MAX_DEVICE_BYTES");
    }
    auto alloc = [&](void** p, size_t b) -> tf_status {
        hipError_t e = hipMalloc(p, b);
        if (e == hipErrorOutOfMemory) return fail(TF_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
        if (e != hipSuccess) return fail(TF_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
        return TF_OK;
    };
    tf_status st = TF_OK;
    if (st == TF_OK) st = alloc(&s->state, state_b);
    if (st == TF_OK) st = alloc(&s->spec, spec_b);
    const int ns[3] = {grid->nx, grid->ny, grid->nz};
    for (int a = 0; a < 3 && st == TF_OK; ++a) st = alloc(&s->tw[a], 2 * s->esize * ns[a]);
    if (st == TF_OK) st = alloc((void**)&s->partials, s->npartials * sizeof(double));
    if (st == TF_OK) st = alloc((void**)&s->results, 8 * sizeof(double));
    if (st == TF_OK) st = alloc(&s->dcbuf, dc_b);
    if (st != TF_OK) {
        free_all(s);
        delete s;
        return st;
    }
    hipError_t e = hipMemsetAsync(s->state, 0, state_b, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->spec, 0, spec_b, s->stream);
    for (int a = 0; a < 3 && e == hipSuccess; ++a) e = upload_twiddles(s->tw[a], ns[a], precision, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        free_all(s);
        delete s;
        return fail(TF_EDEVICE, std::string("initialising solver: ") + hipGetErrorString(e));
    }
    *out = s;
    return TF_OK;
}

tf_status tf_destroy(tf_solver* s) {
    if (!s) return TF_OK;
    hipError_t e = hipStreamSynchronize(s->stream);
    free_all(s);
    delete s;
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("tf_destroy: ") + hipGetErrorString(e));
    return TF_OK;
}

tf_status tf_set_fields(tf_solver* s, const void* src, int32_t src_on_device, double t) {
    if (!s || !src) return fail(TF_EINVAL, "solver and src must not be NULL");
    if (!std::isfinite(t)) return fail(TF_EINVAL, "t must be finite");
    const size_t b = 6 * (size_t)s->cells * s->esize;
    TF_HIP(hipMemcpyAsync(s->state, src, b, src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          s->stream));
    if (!src_on_device) TF_HIP(hipStreamSynchronize(s->stream));
    s->t = t;
    s->project_b_next = false;
    return TF_OK;
}

tf_status tf_get_fields(tf_solver* s, void* dst, int32_t dst_on_device) {
    if (!s || !dst) return fail(TF_EINVAL, "solver and dst must not be NULL");
    const size_t b = 6 * (size_t)s->cells * s->esize;
    TF_HIP(hipMemcpyAsync(dst, s->state, b, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          s->stream));
    if (!dst_on_device) TF_HIP(hipStreamSynchronize(s->stream));
    return TF_OK;
}

tf_status tf_state_ptr(tf_solver* s, void** dev_ptr) {
    if (!s || !dev_ptr) return fail(TF_EINVAL, "solver and dev_ptr must not be NULL");
    *dev_ptr = s->state;
    return TF_OK;
}

tf_status tf_set_pulse(tf_solver* s, const tf_pulse* pulse, tf_pulse_info* info) {
    if (!s) return fail(TF_EINVAL, "solver is NULL");
    tf_status st = validate_pulse(pulse);
    if (st != TF_OK) return st;
    tf_pulse_info g;
    geometry(pulse, &g);
    g.D = s->grid.nx * s->grid.dx;
    g.overlap = g.D < g.D_min ? 1 : 0;
    if (info) *info = g;
    if (!(g.D > pulse->L)) return fail(TF_EDOMAIN, "layer period D = nx dx must exceed the pulse length L");

    tf::PulseDev p = pulse_dev(pulse, g);
    std::vector<double> all;
    size_t spec_len = 0;
    double gnorm = 1.0;
    int nfreq = 0;
    st = pulse_tables(pulse, all, spec_len, gnorm, nfreq);
    if (st != TF_OK) return st;
    if (!all.empty()) {
        if (s->pulse_tab) {
            TF_HIP(hipStreamSynchronize(s->stream));
            TF_HIP(hipFree(s->pulse_tab));
            s->pulse_tab = nullptr;
        }
        TF_HIP(hipMalloc(&s->pulse_tab, all.size() * sizeof(double)));
        TF_HIP(hipMemcpyAsync(s->pulse_tab, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice,
                              s->stream));
        TF_HIP(hipStreamSynchronize(s->stream));
        pulse_dev_tables(p, pulse, static_cast<const double*>(s->pulse_tab), spec_len, gnorm, nfreq);
    }
    tf::GridDev gd = grid_dev(s->grid);
    hipError_t e = timed(s, TF_PASS_INIT, [&] {
        return s->prec == TF_F64 ? tf::launch_init_map<double>(static_cast<double*>(s->state), gd, p, s->stream)
                                 : tf::launch_init_map<float>(static_cast<float*>(s->state), gd, p, s->stream);
    });
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("init kernel: ") + hipGetErrorString(e));
    s->t = 0.0;
    s->project_b_next = true;
    s->have_cutout = true;
    s->R_min = g.R_min;
    s->R_max = g.R_max;
    return TF_OK;
}

tf_status tf_set_cutout(tf_solver* s, double R_min, double R_max) {
    if (!s) return fail(TF_EINVAL, "solver is NULL");
    if (!finite_pos(R_min) || !(R_max > R_min) || !std::isfinite(R_max))
        return fail(TF_EINVAL, "need 0 < R_min < R_max");
    s->R_min = R_min;
    s->R_max = R_max;
    s->have_cutout = true;
    return TF_OK;
}

tf_status tf_advance(tf_solver* s, int64_t nsteps, double dt) {
    if (!s) return fail(TF_EINVAL, "solver is NULL");
    if (nsteps < 0) return fail(TF_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt)) return fail(TF_EINVAL, "dt must be finite");
    auto eager = [&](bool pb) -> tf_status {
        hipError_t e = s->prec == TF_F64 ? one_step<double>(s, dt, pb) : one_step<float>(s, dt, pb);
        if (e != hipSuccess) return fail(TF_EDEVICE, std::string("step: ") + hipGetErrorString(e));
        return TF_OK;
    };
    int64_t i = 0;
    if (s->project_b_next && nsteps > 0) {    // the first step after new fields also removes longitudinal B
        tf_status st = eager(true);
        if (st != TF_OK) return st;
        s->project_b_next = false;
        i = 1;
    }
    // whole graphs of GRAPH_STEPS steps, unless every launch is being timed
    const int64_t graphs = s->prof ? 0 : (nsteps - i) / GRAPH_STEPS;
    if (graphs > 0) {
        tf_status st = s->prec == TF_F64 ? step_graph<double>(s, dt) : step_graph<float>(s, dt);
        if (st != TF_OK) return st;
        for (int64_t r = 0; r < graphs; ++r) TF_HIP(hipGraphLaunch(s->step_exec, s->stream));
        i += graphs * GRAPH_STEPS;
    }
    for (; i < nsteps; ++i) {
        tf_status st = eager(false);
        if (st != TF_OK) return st;
    }
    s->t = s->t + (double)nsteps * dt;
    return TF_OK;
}

tf_status tf_advance_current(tf_solver* s, const void* j, int32_t j_on_device, double dt) {
    if (!s || !j) return fail(TF_EINVAL, "solver and j must not be NULL");
    if (!std::isfinite(dt)) return fail(TF_EINVAL, "dt must be finite");
    const bool fits = s->prec == TF_F64 ? tf::z_current_supported<double>(s->grid.nz)
                                        : tf::z_current_supported<float>(s->grid.nz);
    if (!fits)
        return fail(TF_EUNSUPPORTED, "current steps need nine z columns of " + std::to_string(s->grid.nz) +
                                         " elements in LDS (float64: nz <= 768)");
    const size_t bytes6 = 6 * (size_t)s->cells * s->esize;
    const size_t spec_b = (size_t)s->grid.nz * s->grid.ny * s->nkx * 6 * 2 * s->esize;
    if (!s->jstate || !s->jspec) {
        const size_t have = bytes6 + spec_b + 2 * s->esize * (size_t)(s->grid.nx + s->grid.ny + s->grid.nz);
        if (have + bytes6 + spec_b > device_cap())
            return fail(TF_ENOMEM, "current steps need " + std::to_string(bytes6 + spec_b) +
                                       " more device bytes, above TFOCUS_MAX_DEVICE_BYTES");
        if (!s->jstate) {
            hipError_t e = hipMalloc(&s->jstate, bytes6);
            if (e != hipSuccess) {
                s->jstate = nullptr;
                return fail(e == hipErrorOutOfMemory ? TF_ENOMEM : TF_EDEVICE,
                            std::string("current buffer: ") + hipGetErrorString(e));
            }
            TF_HIP(hipMemsetAsync(static_cast<char*>(s->jstate) + bytes6 / 2, 0, bytes6 / 2, s->stream));
        }
        if (!s->jspec) {
            hipError_t e = hipMalloc(&s->jspec, spec_b);
            if (e != hipSuccess) {
                s->jspec = nullptr;
                return fail(e == hipErrorOutOfMemory ? TF_ENOMEM : TF_EDEVICE,
                            std::string("current spectrum: ") + hipGetErrorString(e));
            }
        }
    }
    TF_HIP(hipMemcpyAsync(s->jstate, j, bytes6 / 2, j_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          s->stream));
    if (!j_on_device) TF_HIP(hipStreamSynchronize(s->stream));
    const bool pb = s->project_b_next;
    hipError_t e = s->prec == TF_F64 ? current_step<double>(s, dt, pb) : current_step<float>(s, dt, pb);
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("current step: ") + hipGetErrorString(e));
    s->project_b_next = false;
    s->t = s->t + dt;
    return TF_OK;
}

tf_status tf_read_focal(tf_solver* s, const tf_window* w, void* dst, int32_t dst_on_device) {
    if (!s || !w || !dst) return fail(TF_EINVAL, "solver, window and dst must not be NULL");
    if (!s->have_cutout) return fail(TF_ESTATE, "no cut-out radii (call tf_set_pulse or tf_set_cutout)");
    if (w->wx <= 0 || w->wy <= 0 || w->wz <= 0) return fail(TF_EINVAL, "window sizes must be > 0");
    if (!std::isfinite(w->cx) || !std::isfinite(w->cy) || !std::isfinite(w->cz))
        return fail(TF_EINVAL, "window centre must be finite");
    const tf_grid& g = s->grid;
    const long ic = (long)std::floor((w->cx - g.x_min) / g.dx + 0.5);
    const long jc = (long)std::floor((w->cy - g.y_min) / g.dy + 0.5);
    const long kc = (long)std::floor((w->cz - g.z_min) / g.dz + 0.5);
    const long j0 = jc - w->wy / 2, j1 = j0 + w->wy - 1, k0 = kc - w->wz / 2, k1 = k0 + w->wz - 1;
    if (!g.replicate_yz && (j0 < 0 || j1 >= g.ny || k0 < 0 || k1 >= g.nz))
        return fail(TF_EINVAL, "window leaves the transverse extent of the grid");
    const size_t bytes = 6 * (size_t)w->wx * w->wy * w->wz * s->esize;
    void* out = dst;
    if (!dst_on_device) {
        if (s->scratch_bytes < bytes) {
            if (s->scratch_out) {
                TF_HIP(hipStreamSynchronize(s->stream));
                TF_HIP(hipFree(s->scratch_out));
                s->scratch_out = nullptr;
                s->scratch_bytes = 0;
            }
            TF_HIP(hipMalloc(&s->scratch_out, bytes));
            s->scratch_bytes = bytes;
        }
        out = s->scratch_out;
    }
    tf::GridDev gd = grid_dev(s->grid);
    hipError_t e = timed(s, TF_PASS_READOUT, [&] {
        return s->prec == TF_F64
                   ? tf::launch_readout<double>(static_cast<const double*>(s->state), static_cast<double*>(out), gd,
                                                w->wx, w->wy, w->wz, ic, jc, kc, s->t, s->R_min, s->R_max, s->stream)
                   : tf::launch_readout<float>(static_cast<const float*>(s->state), static_cast<float*>(out), gd,
                                               w->wx, w->wy, w->wz, ic, jc, kc, s->t, s->R_min, s->R_max, s->stream);
    });
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("readout kernel: ") + hipGetErrorString(e));
    if (!dst_on_device) {
        TF_HIP(hipMemcpyAsync(dst, out, bytes, hipMemcpyDeviceToHost, s->stream));
        TF_HIP(hipStreamSynchronize(s->stream));
    }
    return TF_OK;
}

tf_status tf_diagnostics(tf_solver* s, double* energy, double* max_div_e, double* max_div_b) {
    if (!s) return fail(TF_EINVAL, "solver is NULL");
    hipError_t e;
    const size_t n = 6 * (size_t)s->cells;
    e = s->prec == TF_F64 ? tf::launch_sumsq<double>(static_cast<const double*>(s->state), n, s->partials, tf::SUMSQ_BLOCKS, s->stream)
                          : tf::launch_sumsq<float>(static_cast<const float*>(s->state), n, s->partials, tf::SUMSQ_BLOCKS, s->stream);
    if (e == hipSuccess) e = tf::launch_reduce(s->partials, tf::SUMSQ_BLOCKS, 1, 0, 0, s->results, s->stream);
    if (e == hipSuccess)
        e = s->prec == TF_F64 ? forward_xy<double>(s, TF_PASS_OTHER, TF_PASS_OTHER)
                              : forward_xy<float>(s, TF_PASS_OTHER, TF_PASS_OTHER);
    int nb = 0;
    if (e == hipSuccess) {
        tf::StepParams p = step_params(s->grid, 0.0, false, s->zvariant);
        e = s->prec == TF_F64 ? tf::launch_z_pass<double>(s->spec, s->tw[2], p, s->rm, tf::Z_DIAG, s->partials, s->dcbuf,
                                                          &nb, s->fast, tf::Batch{}, s->stream)
                              : tf::launch_z_pass<float>(s->spec, s->tw[2], p, s->rm, tf::Z_DIAG, s->partials, s->dcbuf,
                                                         &nb, s->fast, tf::Batch{}, s->stream);
    }
    for (int q = 0; q < 4 && e == hipSuccess; ++q) e = tf::launch_reduce(s->partials, nb, 4, q, 1, s->results + 1 + q, s->stream);
    double h[5] = {0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, s->results, sizeof(h), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("diagnostics: ") + hipGetErrorString(e));
    if (energy) *energy = h[0];
    if (max_div_e) *max_div_e = h[3] > 0.0 ? h[1] / h[3] : 0.0;
    if (max_div_b) *max_div_b = h[4] > 0.0 ? h[2] / h[4] : 0.0;
    if (!std::isfinite(h[0])) return fail(TF_ENONFINITE, "field energy is not finite");
    return TF_OK;
}

tf_status tf_advance_diagnosed(tf_solver* s, int64_t nsteps, double dt, double* energy, double* max_div_e,
                               double* max_div_b) {
    if (!s) return fail(TF_EINVAL, "solver is NULL");
    if (nsteps < 1) return fail(TF_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(dt)) return fail(TF_EINVAL, "dt must be finite");
    if (nsteps > 1) {
        tf_status st = tf_advance(s, nsteps - 1, dt);
        if (st != TF_OK) return st;
    }
    int nb = 0;
    const bool pb = s->project_b_next;
    hipError_t e = s->prec == TF_F64 ? one_step<double>(s, dt, pb, &nb) : one_step<float>(s, dt, pb, &nb);
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("diagnosed step: ") + hipGetErrorString(e));
    s->project_b_next = false;
    s->t = s->t + dt;
    const int nz_blocks = nb - s->grid.ny;
    e = tf::launch_reduce(s->partials + 4L * nb, nz_blocks, 1, 0, 0, s->results, s->stream);
    for (int q = 0; q < 4 && e == hipSuccess; ++q) e = tf::launch_reduce(s->partials, nb, 4, q, 1, s->results + 1 + q, s->stream);
    double h[5] = {0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, s->results, sizeof(h), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("diagnostics: ") + hipGetErrorString(e));
    // Parseval: the updated coefficients carry the 1/(nx ny nz) of the inverse transform
    const double en = h[0] * (double)s->cells;
    if (energy) *energy = en;
    if (max_div_e) *max_div_e = h[3] > 0.0 ? h[1] / h[3] : 0.0;
    if (max_div_b) *max_div_b = h[4] > 0.0 ? h[2] / h[4] : 0.0;
    if (!std::isfinite(en)) return fail(TF_ENONFINITE, "field energy is not finite");
    return TF_OK;
}

tf_status tf_time(const tf_solver* s, double* t) {
    if (!s || !t) return fail(TF_EINVAL, "solver and t must not be NULL");
    *t = s->t;
    return TF_OK;
}

tf_status tf_profile(tf_solver* s, int32_t enable) {
    if (!s) return fail(TF_EINVAL, "solver is NULL");
    if (enable) {
        TF_HIP(hipStreamSynchronize(s->stream));
        s->rec_kind.clear();
    }
    s->prof = enable != 0;
    return TF_OK;
}

tf_status tf_profile_read(tf_solver* s, double* ms_total, int64_t* launches) {
    if (!s) return fail(TF_EINVAL, "solver is NULL");
    TF_HIP(hipStreamSynchronize(s->stream));
    double ms[TF_NPASS] = {0};
    int64_t cnt[TF_NPASS] = {0};
    for (size_t i = 0; i < s->rec_kind.size(); ++i) {
        float m = 0.0f;
        TF_HIP(hipEventElapsedTime(&m, s->evpool[2 * i], s->evpool[2 * i + 1]));
        ms[s->rec_kind[i]] += m;
        cnt[s->rec_kind[i]] += 1;
    }
    for (int k = 0; k < TF_NPASS; ++k) {
        if (ms_total) ms_total[k] = ms[k];
        if (launches) launches[k] = cnt[k];
    }
    return TF_OK;
}

tf_status tf_get_grid(const tf_solver* s, tf_grid* grid) {
    if (!s || !grid) return fail(TF_EINVAL, "solver and grid must not be NULL");
    *grid = s->grid;
    return TF_OK;
}

}  // extern "C"
