// Host-side helpers shared by the solver, the batch and the tuner: error
// reporting, argument validation, pulse geometry (Sec. II.B-II.C), the
// sampled spectrum, twiddle tables and the device pulse descriptor.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tfocus.h"
#include "kernels.h"

namespace tf {
namespace host {

// Last error of the calling thread (tf_last_error).
std::string& last_error();

inline tf_status fail(tf_status st, const std::string& msg) {
    last_error() = msg;
    return st;
}

#define TF_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::tf::host::fail(TF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline bool length_ok(int n) {
    return n >= 8 && n <= 1024 && tf::fft_length_supported(n);
}

inline bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// ---- pulse geometry (host, float64) ----

// F(theta0) = int_0^pi sin(a) exp(-2 a^2 / theta0^2) da by composite Simpson
// on [0, min(pi, 12 theta0)] (the integrand is below e^-288 beyond).
inline double F_gauss(double t0) {
    const double b = std::fmin(M_PI, 12.0 * t0);
    const int n = 1 << 20;
    const double h = b / n;
    auto f = [&](double a) { return std::sin(a) * std::exp(-2.0 * a * a / (t0 * t0)); };
    double s = f(0.0) + f(b);
    for (int i = 1; i < n; ++i) s += (i & 1 ? 4.0 : 2.0) * f(i * h);
    return s * h / 3.0;
}

inline tf_status validate_pulse(const tf_pulse* p) {
    if (!p) return fail(TF_EINVAL, "pulse is NULL");
    if (p->envelope < 0 || p->envelope > 2) return fail(TF_EINVAL, "unknown envelope");
    if (p->transverse < 0 || p->transverse > 1) return fail(TF_EINVAL, "unknown transverse profile");
    if (p->polarization < 0 || p->polarization > 1) return fail(TF_EINVAL, "unknown polarization");
    if (!finite_pos(p->wavelength)) return fail(TF_EINVAL, "wavelength must be > 0");
    if (!finite_pos(p->L)) return fail(TF_EINVAL, "L must be > 0");
    if (!finite_pos(p->R0) || !(p->R0 - 0.5 * p->L > 0.0)) return fail(TF_EINVAL, "need R0 > L/2 > 0");
    if (!(p->theta > 0.0) && !finite_pos(p->f_number)) return fail(TF_EINVAL, "need theta > 0 or f_number > 0");
    if (p->theta > 0.0 && !(p->theta < M_PI)) return fail(TF_EINVAL, "theta must be < pi");
    if (p->transverse == TF_TS_FLATTOP && !finite_pos(p->eps)) return fail(TF_EINVAL, "eps must be > 0");
    if (!std::isfinite(p->P0) || p->P0 < 0.0) return fail(TF_EINVAL, "P0 must be >= 0");
    if (p->envelope == TF_ENV_GAUSS && !finite_pos(p->ncycles)) return fail(TF_EINVAL, "ncycles must be > 0");
    if (p->envelope == TF_ENV_SPECTRAL) {
        if (p->nfreq < 1 || p->nfreq > 4096) return fail(TF_EINVAL, "nfreq must be in [1, 4096]");
        if (!finite_pos(p->bandwidth)) return fail(TF_EINVAL, "bandwidth must be > 0");
        if (!std::isfinite(p->gdd) || !std::isfinite(p->tod)) return fail(TF_EINVAL, "chirp must be finite");
    }
    if (!std::isfinite(p->cep) || !std::isfinite(p->pol_angle) || !std::isfinite(p->ellipticity))
        return fail(TF_EINVAL, "phase/polarisation parameters must be finite");
    if (p->polarization == TF_POL_RADIAL && p->ellipticity != 0.0)
        return fail(TF_EINVAL, "radial polarisation takes no ellipticity");
    if (p->nbumps < 0 || p->nbumps > 1024) return fail(TF_EINVAL, "nbumps must be in [0, 1024]");
    if (p->nbumps > 0 && !p->bumps) return fail(TF_EINVAL, "bumps is NULL");
    for (int i = 0; i < p->nbumps; ++i) {
        const double* b = p->bumps + 4 * i;
        if (!std::isfinite(b[0]) || !std::isfinite(b[1]) || !std::isfinite(b[2]) || !finite_pos(b[3]))
            return fail(TF_EINVAL, "phase bumps need finite centres and amplitudes and widths > 0");
    }
    return TF_OK;
}

inline double theta_of(const tf_pulse* p) {
    return p->theta > 0.0 ? p->theta : std::atan(1.0 / (2.0 * p->f_number));
}

inline void geometry(const tf_pulse* p, tf_pulse_info* g) {
    std::memset(g, 0, sizeof(*g));
    const double th = theta_of(p);
    g->theta = th;
    g->L = p->L;
    g->R_min = p->R0 - 0.5 * p->L;
    g->R_max = p->R0 + 0.5 * p->L;
    if (p->transverse == TF_TS_FLATTOP) {
        g->A = std::sqrt(4.0 * p->P0 / (1.0 - std::cos(th)));
        g->alpha_max = th + 0.5 * p->eps;
    } else {
        g->A = std::sqrt(4.0 * p->P0 / F_gauss(th));
        g->alpha_max = 0.5 * M_PI;
    }
    const double s = std::sin(th);
    g->D_min = -g->R_min * std::cos(th) + std::sqrt(g->R_max * g->R_max - g->R_min * g->R_min * s * s);
}

// Spectral samples {w, a, phi} of the sampled Gaussian spectrum and the
// normalisation max |g| over zeta_j = j lambda / 128 inside the window.
inline void spectral_table(const tf_pulse* p, std::vector<double>& tab, double& gnorm) {
    const int M = p->nfreq;
    const double w0 = 2.0 * M_PI / p->wavelength;
    const double dl = p->bandwidth;
    const double X = 4.0;
    tab.clear();
    for (int m = 0; m < M; ++m) {
        const double x = -X + (m + 0.5) * (2.0 * X / M);
        const double w = w0 * (1.0 + dl * x);
        if (!(w > 0.0)) continue;
        const double u = (w - w0) / (dl * w0), v = (w + w0) / (dl * w0);
        const double a = std::exp(-(u * u)) - std::exp(-(v * v));
        const double dw = w - w0;
        const double phi = p->gdd * dw * dw / 2.0 + p->tod * dw * dw * dw / 6.0;
        tab.push_back(w);
        tab.push_back(a);
        tab.push_back(phi);
    }
    const double h = p->wavelength / 128.0;
    const long jmax = (long)std::floor(0.5 * p->L / h);
    gnorm = 0.0;
    const int K = (int)(tab.size() / 3);
    for (long j = -jmax; j <= jmax; ++j) {
        const double z = j * h;
        double acc = 0.0;
        for (int m = 0; m < K; ++m) acc += tab[3 * m + 1] * std::cos(p->cep + 0.5 * M_PI + tab[3 * m + 2] - tab[3 * m] * z);
        gnorm = std::fmax(gnorm, std::fabs(acc));
    }
}

// Device form of the sampled spectrum: the kept samples are uniformly spaced
// (w_m = w0 + m dw), so sum_m a_m exp(i (phi_m - w_m zeta)) is
// exp(-i w0 zeta) times a polynomial in exp(-i dw zeta) with coefficients
// c_m = a_m exp(i phi_m).  Layout {w0, dw, re c_0, im c_0, ...}.
inline std::vector<double> spectral_device_table(const tf_pulse* p, const std::vector<double>& tab) {
    const int K = (int)(tab.size() / 3);
    const double w0 = 2.0 * M_PI / p->wavelength;
    std::vector<double> d(2 + 2 * K);
    d[0] = K > 0 ? tab[0] : 0.0;
    d[1] = w0 * p->bandwidth * (2.0 * 4.0 / p->nfreq);      // w0 delta (2X / M), X = 4
    for (int m = 0; m < K; ++m) {
        d[2 + 2 * m] = tab[3 * m + 1] * std::cos(tab[3 * m + 2]);
        d[3 + 2 * m] = tab[3 * m + 1] * std::sin(tab[3 * m + 2]);
    }
    return d;
}

inline std::vector<double> twiddle_table(int n) {
    std::vector<double> t(2 * n);
    for (int e = 0; e < n; ++e) {
        const double a = 2.0 * M_PI * (double)e / (double)n;
        t[2 * e] = std::cos(a);
        t[2 * e + 1] = -std::sin(a);
    }
    return t;
}

inline size_t device_cap() {
    const char* s = std::getenv("TFOCUS_MAX_DEVICE_BYTES");
    if (!s || !*s) return (size_t)-1;
    return (size_t)std::strtoull(s, nullptr, 10);
}


inline hipError_t upload_twiddles(void* dst, int n, int prec, hipStream_t st) {
    std::vector<double> t = twiddle_table(n);
    hipError_t e;
    if (prec == TF_F64) {
        e = hipMemcpyAsync(dst, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, st);
    } else {
        std::vector<float> f(t.size());
        for (size_t i = 0; i < t.size(); ++i) f[i] = (float)t[i];
        e = hipMemcpyAsync(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e;
    }
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

// Host form of everything the device descriptor points to: the spectral
// table (when the envelope is spectral) followed by the phase bumps.
// spec_len receives the spectral part's length (0 without one); gnorm and
// nfreq as the spectral table gives them.
inline tf_status pulse_tables(const tf_pulse* pulse, std::vector<double>& all, size_t& spec_len, double& gnorm,
                              int& nfreq) {
    all.clear();
    spec_len = 0;
    gnorm = 1.0;
    nfreq = 0;
    if (pulse->envelope == TF_ENV_SPECTRAL) {
        std::vector<double> tab;
        spectral_table(pulse, tab, gnorm);
        if (!(gnorm > 0.0) || tab.empty()) return fail(TF_EINVAL, "spectral pulse has no samples above w = 0");
        all = spectral_device_table(pulse, tab);
        spec_len = all.size();
        nfreq = (int)(tab.size() / 3);
    }
    all.insert(all.end(), pulse->bumps, pulse->bumps + 4 * (size_t)pulse->nbumps);
    return TF_OK;
}

// Points the descriptor at a device copy of pulse_tables' output.
inline void pulse_dev_tables(PulseDev& p, const tf_pulse* pulse, const double* dev, size_t spec_len, double gnorm,
                             int nfreq) {
    if (pulse->envelope == TF_ENV_SPECTRAL) {
        p.spec = dev;
        p.nfreq = nfreq;
        p.gnorm = gnorm;
    }
    p.nbumps = pulse->nbumps;
    p.bumps = pulse->nbumps > 0 ? dev + spec_len : nullptr;
}

// Device pulse descriptor; the spectral table (nfreq x {w, a, phi}) must be
// uploaded by the caller to tab_dev when the envelope is spectral.
inline PulseDev pulse_dev(const tf_pulse* pulse, const tf_pulse_info& g) {
    PulseDev p{};
    p.envelope = pulse->envelope;
    p.transverse = pulse->transverse;
    p.polarization = pulse->polarization;
    p.lambda = pulse->wavelength;
    p.R0 = pulse->R0;
    p.L = pulse->L;
    p.ncycles = pulse->ncycles;
    p.theta = g.theta;
    p.eps = pulse->eps;
    p.A = g.A;
    p.alpha_max = g.alpha_max;
    p.cep = pulse->cep;
    p.gnorm = 1.0;
    if (pulse->polarization == TF_POL_RADIAL) {
        p.nparts = 1;
        p.amp[0] = 1.0;
        p.d[0][0] = 1.0; p.d[0][1] = 0.0; p.d[0][2] = 0.0;
        p.phase_off[0] = 0.0;
        p.phase_off[1] = 0.0;
    } else {
        const double c = std::cos(pulse->pol_angle), sn = std::sin(pulse->pol_angle);
        const double e = pulse->ellipticity;
        const double nrm = std::sqrt(1.0 + e * e);
        p.nparts = e != 0.0 ? 2 : 1;
        p.amp[0] = 1.0 / nrm;
        p.d[0][0] = 0.0; p.d[0][1] = c; p.d[0][2] = sn;
        p.phase_off[0] = 0.0;
        p.amp[1] = e / nrm;
        p.d[1][0] = 0.0; p.d[1][1] = -sn; p.d[1][2] = c;
        p.phase_off[1] = 0.5 * M_PI;
    }
    for (int k = 0; k < 2; ++k) {
        p.cph[k] = std::cos(p.cep + p.phase_off[k] + 0.5 * M_PI);
        p.sph[k] = std::sin(p.cep + p.phase_off[k] + 0.5 * M_PI);
    }
    return p;
}

inline GridDev grid_dev(const tf_grid& s) {
    GridDev g;
    g.nx = s.nx; g.ny = s.ny; g.nz = s.nz;
    g.dx = s.dx; g.dy = s.dy; g.dz = s.dz;
    g.x_min = s.x_min; g.y_min = s.y_min; g.z_min = s.z_min;
    g.rep_yz = s.replicate_yz;
    return g;
}

inline StepParams step_params(const tf_grid& g, double dt, bool project_b, int zvariant) {
    StepParams p;
    p.nx = g.nx; p.ny = g.ny; p.nz = g.nz; p.nkx = nkx_of(g.nx);
    p.kfx = 2.0 * M_PI / (g.nx * g.dx);
    p.kfy = 2.0 * M_PI / (g.ny * g.dy);
    p.kfz = 2.0 * M_PI / (g.nz * g.dz);
    p.cdt = dt;
    p.scale = 1.0 / ((double)g.nx * (double)g.ny * (double)g.nz);
    p.project_b = project_b ? 1 : 0;
    p.zvariant = zvariant;
    // largest phase c |k| dt of the grid (signed modes reach n/2 per axis);
    // up to 8 rad z variant 10 builds its phase factors in float32
    const double kmax = std::sqrt(std::pow(p.kfx * (g.nx / 2), 2) + std::pow(p.kfy * (g.ny / 2), 2) +
                                  std::pow(p.kfz * (g.nz / 2), 2));
    p.phase32 = std::fabs(p.cdt) * kmax <= 8.0 ? 1 : 0;
    return p;
}

inline tf_status validate_grid(const tf_grid* grid) {
    if (!grid) return fail(TF_EINVAL, "grid is NULL");
    if (grid->nx % 2 != 0) return fail(TF_EINVAL, "nx must be even");
    if (grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0) return fail(TF_EINVAL, "grid sizes must be > 0");
    if (!finite_pos(grid->dx) || !finite_pos(grid->dy) || !finite_pos(grid->dz))
        return fail(TF_EINVAL, "spacings must be finite and > 0");
    if (!std::isfinite(grid->x_min) || !std::isfinite(grid->y_min) || !std::isfinite(grid->z_min))
        return fail(TF_EINVAL, "grid origin must be finite");
    if (grid->replicate_yz != 0 && grid->replicate_yz != 1) return fail(TF_EINVAL, "replicate_yz must be 0 or 1");
    for (int n : {grid->nx, grid->ny, grid->nz})
        if (!length_ok(n))
            return fail(TF_EUNSUPPORTED, "axis length " + std::to_string(n) +
                                             " unsupported (see tf_supported_length)");
    return TF_OK;
}

// Kernel shape choices for one grid (row blocking, fast kernels, z variant);
// from the tuned plan file when it has an entry, else defaults, then
// environment overrides.
struct KernelPlan {
    int row_block = 8;
    bool fast = true;
    int zvariant = 0;
    int ystrip = 64;       // columns per strip of the fast y kernel (64 or 32)
    int yarg() const { return fast ? ystrip : 0; }
};
KernelPlan plan_for(const tf_grid& g, int precision);

// Whether the fast float32 kernels can address a grid with this row blocking
// (the fast z kernel's 32-bit strip offsets, z_fast_offsets_fit).
inline bool fast_offsets_fit(const tf_grid& g, int row_block, int precision) {
    const size_t cb = precision == TF_F64 ? 16 : 8;
    return z_fast_offsets_fit(g.nx, g.nz, row_block, cb);
}

// Pass sequence of one step on a set of same-shape instances.
template <typename T>
hipError_t step_passes(void* state, void* spec, void* const* tw, const tf_grid& g, const RowMap& rm,
                       const KernelPlan& kp, double dt, bool project_b, Batch bt, hipStream_t st) {
    hipError_t e = launch_x_forward<T>(static_cast<const T*>(state), spec, tw[0], g.nx, g.ny, g.nz, rm, bt, st);
    if (e != hipSuccess) return e;
    e = launch_y_pass<T>(spec, tw[1], g.nx, g.ny, g.nz, -1, rm, kp.yarg(), bt, st);
    if (e != hipSuccess) return e;
    StepParams p = step_params(g, dt, project_b, kp.zvariant);
    if (bt.cdt) p.phase32 = 0;          // per-instance time steps: the phase bound is not known here
    e = launch_z_pass<T>(spec, tw[2], p, rm, Z_STEP, nullptr, nullptr, nullptr, kp.fast, bt, st);
    if (e != hipSuccess) return e;
    e = launch_y_pass<T>(spec, tw[1], g.nx, g.ny, g.nz, +1, rm, kp.yarg(), bt, st);
    if (e != hipSuccess) return e;
    return launch_x_inverse<T>(spec, static_cast<T*>(state), tw[0], g.nx, g.ny, g.nz, rm, bt, st);
}

}  // namespace host
}  // namespace tf
