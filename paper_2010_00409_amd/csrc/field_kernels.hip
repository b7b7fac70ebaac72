// Pulse initialisation with mapping into the periodic layer, focal-window
// cut-out and deterministic reductions.  Built with -ffp-contract=off so the
// float64 geometry (radii, angles, cut-out decisions) rounds like a plain
// evaluation of the same expressions.
#include "kernels.h"

namespace tf {

// ---------------------------------------------------------------- profiles
// Transverse profile: flat-top of Eq. (5) (first window half-open) or the
// Gaussian exp(-a^2/theta^2) of Sec. III.B.1 restricted to a <= pi/2.
__device__ double u_ts(double alpha, const PulseDev& p) {
    if (p.transverse == 0) {
        const double lo = p.theta - 0.5 * p.eps, hi = p.theta + 0.5 * p.eps;
        if (alpha < lo) return 1.0;
        if (alpha <= hi) {
            const double c = cos(M_PI * (alpha - p.theta + 0.5 * p.eps) / (2.0 * p.eps));
            return c * c;
        }
        return 0.0;
    }
    if (alpha <= 0.5 * M_PI) return exp(-(alpha * alpha) / (p.theta * p.theta));
    return 0.0;
}

// Longitudinal profile with carrier, zeta inside [-L/2, L/2] (checked by the
// caller), for the cos^2 envelope of Eq. (7) and the Gaussian envelope of
// Sec. III.B.1.
__device__ double u_l_closed(double zeta, double phase, const PulseDev& p) {
    if (p.envelope == 0) {
        const double c = cos(M_PI * zeta / p.L);
        return sin(2.0 * M_PI * zeta / p.lambda - phase) * (c * c);
    }
    const double nl = p.ncycles * p.lambda;
    return sin(2.0 * M_PI * zeta / p.lambda - phase) * exp(-zeta * zeta * log(4.0) / (nl * nl));
}

// Sampled spectrum: S(zeta) = sum_m a_m exp(i (phi_m - w_m zeta)), evaluated
// as exp(-i w0 zeta) P(exp(-i dw zeta)) with P(z) = sum_m c_m z^m by Horner's
// rule (|z| = 1, so the rounding stays at a few ulps of sum |c_m|).  The
// profile of a part with carrier phase ph is Re[exp(i (ph + pi/2)) S] / gnorm.
__device__ void spectral_sum(double zeta, const PulseDev& p, double& sr, double& si) {
    const double* c = p.spec + 2;
    const int K = p.nfreq;
    double zs, zc, es, ec;
    sincos(-p.spec[1] * zeta, &zs, &zc);
    sincos(-p.spec[0] * zeta, &es, &ec);
    double pr = c[2 * (K - 1)], pim = c[2 * (K - 1) + 1];
    for (int m = K - 2; m >= 0; --m) {
        const double tr = pr * zc - pim * zs;
        const double ti = pr * zs + pim * zc;
        pr = c[2 * m] + tr;
        pim = c[2 * m + 1] + ti;
    }
    sr = pr * ec - pim * es;
    si = pr * es + pim * ec;
}

// Wavefront phase of the direction (alpha, azimuth): a sum of Gaussian bumps
// over the angular position (ay, az) = alpha (y, z) / rho (Sec. III.B.3).
__device__ double bump_phase(double alpha, double y, double z, double rho, const PulseDev& p) {
    const double ay = rho > 0.0 ? alpha * y / rho : 0.0;
    const double az = rho > 0.0 ? alpha * z / rho : 0.0;
    double ph = 0.0;
    for (int i = 0; i < p.nbumps; ++i) {
        const double* bp = p.bumps + 4 * i;
        const double dy = ay - bp[0], dz = az - bp[1];
        ph += bp[2] * exp(-(dy * dy + dz * dz) / (bp[3] * bp[3]));
    }
    return ph;
}

// Adds the unmapped pulse at physical point (x, y, z) to e, b.
__device__ void add_pulse(double x, double y, double z, const PulseDev& p, double* e, double* b) {
    const double R = sqrt(x * x + y * y + z * z);
    const double zeta = R - p.R0;
    if (!(zeta >= -0.5 * p.L && zeta <= 0.5 * p.L)) return;
    const double rho = sqrt(y * y + z * z);
    const double alpha = atan2(rho, -x);                    // angle from the -x axis
    if (!(alpha <= p.alpha_max)) return;
    const double ts = u_ts(alpha, p);
    double sr = 0.0, si = 0.0;
    if (p.envelope == 2) spectral_sum(zeta, p, sr, si);     // shared by both polarisation parts
    // the perturbation adds to every part's carrier phase, as the CEP does
    const double dph = p.nbumps > 0 ? bump_phase(alpha, y, z, rho, p) : 0.0;
    double cb = 1.0, sb = 0.0;
    if (p.nbumps > 0 && p.envelope == 2) sincos(dph, &sb, &cb);
    for (int k = 0; k < p.nparts; ++k) {
        const double ul = p.envelope == 2
                              ? ((p.cph[k] * cb - p.sph[k] * sb) * sr - (p.sph[k] * cb + p.cph[k] * sb) * si) / p.gnorm
                              : u_l_closed(zeta, p.cep + p.phase_off[k] + dph, p);
        const double u = p.A / R * ul * ts;
        const double* d = p.d[k];
        // s1 ~ d x R, s0 ~ R x (d x R)
        const double c1x = d[1] * z - d[2] * y, c1y = d[2] * x - d[0] * z, c1z = d[0] * y - d[1] * x;
        const double n1 = sqrt(c1x * c1x + c1y * c1y + c1z * c1z);
        if (!(n1 > 0.0)) continue;
        const double c0x = y * c1z - z * c1y, c0y = z * c1x - x * c1z, c0z = x * c1y - y * c1x;
        const double au = p.amp[k] * u;
        const double i1 = 1.0 / n1, i0 = 1.0 / (n1 * R);
        e[0] += au * c0x * i0; e[1] += au * c0y * i0; e[2] += au * c0z * i0;
        b[0] += au * c1x * i1; b[1] += au * c1y * i1; b[2] += au * c1z * i1;
    }
}

// One thread per layer node: sum of the pulse over the preimages x + n D,
// n ascending (Eq. (13) inverted; overlapping replicas superpose); with
// transverse replication also over y + m Dy, z + l Dz (l, then m ascending
// outside the x preimages).
template <typename T>
__global__ __launch_bounds__(256) void k_init_map(T* __restrict__ state, GridDev g, PulseDev p) {
    const long cells = (long)g.nx * g.ny * g.nz;
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= cells) return;
    const int i = (int)(id % g.nx);
    const int j = (int)((id / g.nx) % g.ny);
    const int k = (int)(id / ((long)g.nx * g.ny));
    const double D = g.nx * g.dx;
    const double xt = g.x_min + i * g.dx;
    const double y = g.y_min + j * g.dy;
    const double z = g.z_min + k * g.dz;
    const double Rmax = p.R0 + 0.5 * p.L;
    double e[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
    const long n0 = (long)floor((-Rmax - xt) / D) - 1;
    const long n1 = (long)ceil((Rmax - xt) / D) + 1;
    long m0 = 0, m1 = 0, l0 = 0, l1 = 0;
    const double Dy = g.ny * g.dy, Dz = g.nz * g.dz;
    if (g.rep_yz) {
        m0 = (long)floor((-Rmax - y) / Dy) - 1;
        m1 = (long)ceil((Rmax - y) / Dy) + 1;
        l0 = (long)floor((-Rmax - z) / Dz) - 1;
        l1 = (long)ceil((Rmax - z) / Dz) + 1;
    }
    for (long l = l0; l <= l1; ++l)
        for (long m = m0; m <= m1; ++m) {
            const double yy = g.rep_yz ? y + m * Dy : y, zz = g.rep_yz ? z + l * Dz : z;
            if (yy * yy + zz * zz <= Rmax * Rmax)
                for (long n = n0; n <= n1; ++n) add_pulse(xt + n * D, yy, zz, p, e, b);
        }
    state[0 * cells + id] = T(e[0]);
    state[1 * cells + id] = T(e[1]);
    state[2 * cells + id] = T(e[2]);
    state[3 * cells + id] = T(b[0]);
    state[4 * cells + id] = T(b[1]);
    state[5 * cells + id] = T(b[2]);
}

// ---------------------------------------------------------------- cut-out
// Coordinate of node I along an axis.  When the origin is a node (lo / d an
// integer), the coordinate is the node's integer offset from the origin
// times d, so grids that share the spacing give the very same value to the
// same point, and the cut-out of Eq. (15) decides nodes on its spheres
// (R = L, R = r(t), ...) alike in every such grid.
__device__ double node_coord(long I, double lo, double d) {
    const double o = lo / d, r = rint(o);
    return fabs(o - r) <= 1e-6 ? (double)(I + (long)r) * d : lo + I * d;
}

// I_S(t)(R) of Eq. (15), third case read as "x >= 0 and R > r(t)".
__device__ bool cutout_keep(double x, double y, double z, double t, double Rmin, double Rmax) {
    const double R = sqrt(x * x + y * y + z * z);
    const double L = Rmax - Rmin;
    const double l = -Rmax + t, r = -Rmin + t;
    if (r < 0.0) return !((R >= -l) || (R < -r) || (x > 0.0));
    if (l <= 0.0) return !(((x < 0.0) && (R > L)) || ((x >= 0.0) && (R > r)));
    return !((R <= l) || (R > r) || (x < 0.0));
}

template <typename T>
__global__ __launch_bounds__(256) void k_readout(const T* __restrict__ state, T* __restrict__ out, GridDev g,
                                                 int wx, int wy, int wz, long ic, long jc, long kc,
                                                 double t, double Rmin, double Rmax) {
    const long wn = (long)wx * wy * wz;
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= wn) return;
    const int a = (int)(id % wx), bj = (int)((id / wx) % wy), ck = (int)(id / ((long)wx * wy));
    const long I = ic + a - wx / 2, J = jc + bj - wy / 2, K = kc + ck - wz / 2;
    long ix = I % g.nx;
    if (ix < 0) ix += g.nx;
    long jy = J, kz = K;
    if (g.rep_yz) {
        jy = J % g.ny;
        if (jy < 0) jy += g.ny;
        kz = K % g.nz;
        if (kz < 0) kz += g.nz;
    }
    const double x = node_coord(I, g.x_min, g.dx), y = node_coord(J, g.y_min, g.dy), z = node_coord(K, g.z_min, g.dz);
    const bool keep = cutout_keep(x, y, z, t, Rmin, Rmax);
    const long cells = (long)g.nx * g.ny * g.nz;
    const long src = (kz * g.ny + jy) * g.nx + ix;
    for (int c = 0; c < 6; ++c) out[c * wn + id] = keep ? state[c * cells + src] : T(0);
}

// ---------------------------------------------------------------- reductions
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const T* __restrict__ x, size_t n, double* __restrict__ part) {
    __shared__ double red[4];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double v = double(x[i]);
        acc += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part, int m, int stride, int offset,
                                                int op, double* __restrict__ out) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double v = part[(long)i * stride + offset];
        acc = op == 0 ? acc + v : fmax(acc, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(acc, off);
        acc = op == 0 ? acc + o : fmax(acc, o);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        *out = op == 0 ? ((red[0] + red[1]) + red[2]) + red[3]
                       : fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    }
}

// ---------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_init_map(T* state, const GridDev& g, const PulseDev& p, hipStream_t st) {
    const long cells = (long)g.nx * g.ny * g.nz;
    const unsigned nb = (unsigned)((cells + 255) / 256);
    hipLaunchKernelGGL(k_init_map<T>, dim3(nb), dim3(256), 0, st, state, g, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_readout(const T* state, T* out, const GridDev& g, int wx, int wy, int wz, long ic, long jc,
                          long kc, double t, double R_min, double R_max, hipStream_t st) {
    const long wn = (long)wx * wy * wz;
    const unsigned nb = (unsigned)((wn + 255) / 256);
    hipLaunchKernelGGL(k_readout<T>, dim3(nb), dim3(256), 0, st, state, out, g, wx, wy, wz, ic, jc, kc, t,
                       R_min, R_max);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sumsq(const T* x, size_t n, double* partials, int nb, hipStream_t st) {
    hipLaunchKernelGGL(k_sumsq<T>, dim3(nb), dim3(256), 0, st, x, n, partials);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int m, int stride, int offset, int op, double* out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, partials, m, stride, offset, op, out);
    return hipGetLastError();
}

template hipError_t launch_init_map<float>(float*, const GridDev&, const PulseDev&, hipStream_t);
template hipError_t launch_init_map<double>(double*, const GridDev&, const PulseDev&, hipStream_t);
template hipError_t launch_readout<float>(const float*, float*, const GridDev&, int, int, int, long, long, long,
                                          double, double, double, hipStream_t);
template hipError_t launch_readout<double>(const double*, double*, const GridDev&, int, int, int, long, long,
                                           long, double, double, double, hipStream_t);
template hipError_t launch_sumsq<float>(const float*, size_t, double*, int, hipStream_t);
template hipError_t launch_sumsq<double>(const double*, size_t, double*, int, hipStream_t);

}  // namespace tf
