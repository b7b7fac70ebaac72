// Internal interface between the host engine and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tf {

// Spectral layout: rows of nkx = nx/2 mode slots x 6 components (complex);
// slot 0 packs the x DC and Nyquist planes as F(0) + i F(nx/2).  Row (kz, ky)
// sits at RowMap::row: y is split into blocks of G rows, so rows are ordered
// [ky / G][kz][ky % G]; z neighbours are G rows apart and y neighbours within
// a block are adjacent.
inline int nkx_of(int nx) { return nx / 2; }

// The fast z kernel addresses a strip as a block-uniform 64-bit base plus
// 32-bit byte offsets; they reach (nz - 1) G rows of 6 nkx complex values
// beyond the base (plus one row), which must stay below 4 GiB.
inline bool z_fast_offsets_fit(int nx, int nz, int G, size_t complex_bytes) {
    const unsigned long long rowb = 6ull * (unsigned long long)nkx_of(nx) * complex_bytes;
    return ((unsigned long long)(nz - 1) * (unsigned long long)G + 1ull) * rowb <= (1ull << 32);
}

// Row of (kz, ky) in the spectral array: G = ny keeps rows in natural
// order (kz major); otherwise G, a power of two dividing ny, blocks ky by G
// (rows [ky / G][kz][ky % G]).  The passes compute a row for every element
// they move, so the row is a shift and two masks set up on the host, with
// no division and no branch: ky / G = (ky >> sh) & qmask, ky % G = ky & rmask
// (unblocked: qmask = 0, rmask = all ones).
struct RowMap {
    int ny = 0, nz = 0, G = 0;
    int sh = 0, qmask = 0, rmask = 0;
    RowMap() = default;
    __host__ __device__ RowMap(int ny_, int nz_, int G_) : ny(ny_), nz(nz_), G(G_) {
        if (G >= ny) {
            sh = 0; qmask = 0; rmask = -1;
        } else {
            while ((1 << sh) < G) ++sh;
            qmask = -1; rmask = G - 1;
        }
    }
    __host__ __device__ __forceinline__ long row(int z, int y) const {
        return ((long)((y >> sh) & qmask) * nz + z) * G + (y & rmask);
    }
};

// Row blockings RowMap supports for an axis of ny: ny itself or a power of two dividing ny.
inline bool row_block_ok(int G, int ny) {
    return G == ny || (G > 0 && (G & (G - 1)) == 0 && ny % G == 0);
}

struct StepParams {
    int nx, ny, nz, nkx;
    double kfx, kfy, kfz;    // 2 pi / (n d) per axis
    double cdt;              // c dt
    double scale;            // 1 / (nx ny nz)
    int project_b;           // also remove the longitudinal part of B
    int zvariant;            // shape of the fused float32 z kernel (strip modes, elements per lane, first radix)
    int phase32;             // |c dt| |k|max <= 8: z variant 10 may build the phase in float32
};

enum ZMode { Z_STEP = 0, Z_DIAG = 1, Z_STEP_DIAG = 2 };

// Launch over n same-shape instances (grid y): instance i's state and
// spectrum start sreal resp. sspec elements (of the element type resp.
// complex) after instance 0's; cdt (nullable, n values on the device)
// overrides StepParams::cdt per instance.
struct Batch {
    int n = 1;
    long sreal = 0, sspec = 0;
    const double* cdt = nullptr;
};

// Forward x pass: real state [6][nz][ny][nx] -> spectral (x transformed).
template <typename T> hipError_t launch_x_forward(const T* real, void* spec, const void* tw,
                                                  int nx, int ny, int nz, RowMap rm, Batch bt, hipStream_t st);
// Inverse x pass: spectral -> real state.
template <typename T> hipError_t launch_x_inverse(const void* spec, T* real, const void* tw,
                                                  int nx, int ny, int nz, RowMap rm, Batch bt, hipStream_t st);
// In-place y transform of the spectral array, dir = -1 forward, +1 inverse.
// ystrip: columns per strip of the fast float32 kernel (64 or 32; 64 falls
// back to 32 on rows of 32 (mod 64) slots); 0 forces the generic kernels.
template <typename T> hipError_t launch_y_pass(void* spec, const void* tw, int nx, int ny, int nz,
                                               int dir, RowMap rm, int ystrip, Batch bt, hipStream_t st);
// z pass: Z_STEP = forward z FFT, Eqs. (3)-(4) update, inverse z FFT, in place;
// Z_DIAG = forward z FFT and per-block maxima |k.E|, |k.B|, |E|, |B| into
// partials (4 doubles per block; the packed kx = 0 slot goes through dc, a
// buffer of ny nz 6 complex elements), no store.  *nblocks receives the
// number of 4-wide partials written.  Z_STEP_DIAG = Z_STEP (generic kernel)
// whose blocks also take the diagnostics of the updated spectrum (the next
// state, scaled by 1/(nx ny nz)): the 4-wide maxima as Z_DIAG, then after
// the 4 *nblocks maxima one weighted sum of |coefficient|^2 per z block
// (*nblocks - ny of them; Parseval energy up to the factor nx ny nz).
template <typename T> hipError_t launch_z_pass(void* spec, const void* tw, const StepParams& p,
                                               RowMap rm, int mode, double* partials, void* dc,
                                               int* nblocks, bool fast, Batch bt, hipStream_t st);
template <typename T> int z_diag_blocks(int nx, int ny, int nz);
// z pass of a step with a current (Eqs. (1)-(2)): jspec holds the x- and
// y-transformed current in components 0..2 of the same layout as spec.
// Generic kernel, one mode slot per block, for every nz whose nine columns
// fit the LDS (z_current_supported).
template <typename T> hipError_t launch_z_current(void* spec, const void* jspec, const void* tw,
                                                  const StepParams& p, RowMap rm, hipStream_t st);
template <typename T> bool z_current_supported(int nz);

// Twiddle tables are per axis length: tw[e] = exp(-2 pi i e / n).
bool fft_length_supported(int n);

// ---- field kernels (init + map, cut-out, reductions) ----

struct PulseDev {
    int envelope, transverse, polarization, nfreq;
    double lambda, R0, L, ncycles, theta, eps, A, alpha_max, cep;
    double gnorm;                 // spectral normalisation
    int nparts;                   // 1 or 2 polarisation parts
    double amp[2], d[2][3], phase_off[2];
    double cph[2], sph[2];        // cos, sin of cep + phase_off + pi/2 (spectral carrier phase)
    // spectral only: {w0, dw, then c_m = a_m exp(i phi_m) as re, im} for the
    // nfreq kept samples w_m = w0 + m dw
    const double* spec;
    // wavefront phase bumps {ay, az, amplitude, width} (nbumps of them)
    int nbumps;
    const double* bumps;
};

struct GridDev {
    int nx, ny, nz;
    double dx, dy, dz, x_min, y_min, z_min;
    int rep_yz;                   // y and z are periods of the mapping too
};

template <typename T> hipError_t launch_init_map(T* state, const GridDev& g, const PulseDev& p,
                                                 hipStream_t st);
template <typename T> hipError_t launch_readout(const T* state, T* out, const GridDev& g,
                                                int wx, int wy, int wz, long ic, long jc, long kc,
                                                double t, double R_min, double R_max,
                                                hipStream_t st);
// Sum of squares of n elements into partials[nb] (fixed grid, deterministic).
template <typename T> hipError_t launch_sumsq(const T* x, size_t n, double* partials, int nb,
                                              hipStream_t st);
// Single-block reductions of m partials: op 0 = sum, 1 = max; stride/offset
// select a strided slice (for the 4-wide z-diagnostic partials).
hipError_t launch_reduce(const double* partials, int m, int stride, int offset, int op,
                         double* out, hipStream_t st);

constexpr int SUMSQ_BLOCKS = 1024;

}  // namespace tf
