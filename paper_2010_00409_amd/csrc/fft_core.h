// Device building blocks of the spectral step: complex arithmetic, radix
// 2/3/4/5/7/8 butterflies and a Stockham autosort FFT over sequences held in
// LDS.
//
// Transform convention (the forward transform of the spectral solver,
// Sec. II.A): X[m] = sum_j x[j] w^(m j) with w = exp(DIR 2 pi i / N),
// DIR = -1 forward, +1 inverse (unnormalised).  Twiddles come from a table
// tw[e] = exp(-2 pi i e / N), e in [0, N), built on the host in float64 from
// the exact integer phase and rounded to the element type.
#pragma once
#include <hip/hip_runtime.h>

namespace tf {

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename T> using C2 = typename cplx_of<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { a.x += b.x; a.y += b.y; return a; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename V> __device__ __forceinline__ V cconj(V a) { a.y = -a.y; return a; }
// a * (DIR i): DIR = +1 -> (-y, x); DIR = -1 -> (y, -x)
template <int DIR, typename V> __device__ __forceinline__ V cmul_i(V a) {
    V r;
    if (DIR > 0) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
    return r;
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { a.x *= s; a.y *= s; return a; }

template <typename T> struct Consts;
template <> struct Consts<float> {
    static constexpr float r2 = 0.70710678118654752440f;   // sqrt(2)/2
    static constexpr float r3 = 0.86602540378443864676f;   // sqrt(3)/2
};
template <> struct Consts<double> {
    static constexpr double r2 = 0.70710678118654752440;
    static constexpr double r3 = 0.86602540378443864676;
};

// In-register DFTs of length R; output in natural order v[0..R).
template <typename T, int DIR> __device__ __forceinline__ void dft2(C2<T>* v) {
    C2<T> a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
}

template <typename T, int DIR> __device__ __forceinline__ void dft3(C2<T>* v) {
    C2<T> s = cadd(v[1], v[2]);
    C2<T> d = csub(v[1], v[2]);
    C2<T> m = csub(v[0], cscale(s, T(0.5)));
    C2<T> t = cscale(cmul_i<DIR>(d), Consts<T>::r3);
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, t);
    v[2] = csub(m, t);
}

template <typename T, int DIR> __device__ __forceinline__ void dft4(C2<T>* v) {
    C2<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C2<T> t2 = cadd(v[1], v[3]), t3 = cmul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2); v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3); v[3] = csub(t1, t3);
}

// a + s b, elementwise with fused multiply-adds
template <typename V, typename S> __device__ __forceinline__ V cfma(S s, V b, V a) {
    a.x = fma(s, b.x, a.x); a.y = fma(s, b.y, a.y); return a;
}

// Radix 2 x 4: even outputs are the 4-point DFT of c_k = v_k + v_(k+4); odd
// outputs the 4-point DFT of (v_k - v_(k+4)) w8^k, w8 = exp(DIR 2 pi i / 8).
// w8 and w8^3 are sqrt(2)/2 (1 + DIR i) and sqrt(2)/2 (-1 + DIR i); the
// common factor sqrt(2)/2 is applied in the last additions as fused
// multiply-adds.
template <typename T, int DIR> __device__ __forceinline__ void dft8(C2<T>* v) {
    C2<T> b[4], c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) { b[k] = cadd(v[k], v[k + 4]); c[k] = csub(v[k], v[k + 4]); }
    const T s = Consts<T>::r2;
    const C2<T> u1 = cadd(c[1], cmul_i<DIR>(c[1]));            // c1 w8 / s
    const C2<T> u3 = csub(cmul_i<DIR>(c[3]), c[3]);            // c3 w8^3 / s
    const C2<T> c2 = cmul_i<DIR>(c[2]);                        // c2 w8^2
    const C2<T> t0 = cadd(c[0], c2), t1 = csub(c[0], c2);
    const C2<T> pa = cadd(u1, u3), pb = cmul_i<DIR>(csub(u1, u3));
    dft4<T, DIR>(b);
#pragma unroll
    for (int m = 0; m < 4; ++m) v[2 * m] = b[m];
    v[1] = cfma(s, pa, t0);
    v[5] = cfma(-s, pa, t0);
    v[3] = cfma(s, pb, t1);
    v[7] = cfma(-s, pb, t1);
}

// cos and sin of 2 pi k / R for odd R = 5, 7 and k = 1 .. (R - 1) / 2
// (the real and imaginary parts of the R-th roots of unity).
template <int R> struct OddRoots;
template <> struct OddRoots<5> {
    static constexpr double c[2] = {0.30901699437494742410, -0.80901699437494742410};
    static constexpr double s[2] = {0.95105651629515357212, 0.58778525229247312917};
};
template <> struct OddRoots<7> {
    static constexpr double c[3] = {0.62348980185873353053, -0.22252093395631440429, -0.90096886790241912624};
    static constexpr double s[3] = {0.78183148246802980871, 0.97492791218182360702, 0.43388373911755812048};
};

// Length-R DFT for odd prime R from symmetric pairs: with a_j = x_j + x_{R-j}
// and b_j = x_j - x_{R-j}, X_m = x_0 + sum_j a_j cos(2 pi j m / R)
// + DIR i sum_j b_j sin(2 pi j m / R), and X_{R-m} the same with the sine
// sum negated (m = 1 .. (R - 1) / 2).
template <typename T, int R, int DIR> __device__ __forceinline__ void dft_odd(C2<T>* v) {
    constexpr int H = (R - 1) / 2;
    C2<T> a[H], b[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) { a[j - 1] = cadd(v[j], v[R - j]); b[j - 1] = csub(v[j], v[R - j]); }
    const C2<T> x0 = v[0];
    C2<T> sum = x0;
#pragma unroll
    for (int j = 0; j < H; ++j) sum = cadd(sum, a[j]);
    v[0] = sum;
#pragma unroll
    for (int m = 1; m <= H; ++m) {
        C2<T> re = x0, im{T(0), T(0)};
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const int k = (j * m) % R;                       // angle index of j m, folded to 1 .. H
            const int kk = k <= H ? k : R - k;
            const T cj = T(OddRoots<R>::c[kk - 1]);
            const T sj = T(k <= H ? OddRoots<R>::s[kk - 1] : -OddRoots<R>::s[kk - 1]);
            re.x += cj * a[j - 1].x; re.y += cj * a[j - 1].y;
            im.x += sj * b[j - 1].x; im.y += sj * b[j - 1].y;
        }
        const C2<T> t = cmul_i<DIR>(im);
        v[m] = cadd(re, t);
        v[R - m] = csub(re, t);
    }
}

template <typename T, int R, int DIR> __device__ __forceinline__ void dftR(C2<T>* v) {
    static_assert(R == 2 || R == 3 || R == 4 || R == 5 || R == 7 || R == 8, "radix 2, 3, 4, 5, 7 or 8");
    if constexpr (R == 2) dft2<T, DIR>(v);
    else if constexpr (R == 3) dft3<T, DIR>(v);
    else if constexpr (R == 4) dft4<T, DIR>(v);
    else if constexpr (R == 5 || R == 7) dft_odd<T, R, DIR>(v);
    else dft8<T, DIR>(v);
}

// Radix schedule of a length N = 2^a 3^b 5^c 7^d: radix-8 stages, then one
// radix-4 or radix-2 stage for the rest of the power of two, then radix-3,
// radix-5 and radix-7 stages.
constexpr int log2_part(int n) { int a = 0; while (n % 2 == 0) { n /= 2; ++a; } return a; }
constexpr int log3_part(int n) { int b = 0; while (n % 3 == 0) { n /= 3; ++b; } return b; }
constexpr int logp_part(int n, int p) { int b = 0; while (n % p == 0) { n /= p; ++b; } return b; }
constexpr int ipow(int p, int e) { int r = 1; while (e-- > 0) r *= p; return r; }
template <int N> struct Plan {
    static constexpr int a = log2_part(N);
    static constexpr int b = log3_part(N);
    static constexpr int c5 = logp_part(N, 5);
    static constexpr int c7 = logp_part(N, 7);
    static constexpr int n8 = a / 3;
    static constexpr int rem = a % 3;
    static constexpr int n2 = n8 + (rem ? 1 : 0);
    static constexpr int nst = n2 + b + c5 + c7;
    static constexpr int radix(int s) {
        return s < n8 ? 8 : (s < n2 ? (1 << rem) : (s < n2 + b ? 3 : (s < n2 + b + c5 ? 5 : 7)));
    }
    static_assert(N == (1 << a) * ipow(3, b) * ipow(5, c5) * ipow(7, c7), "N must be 2^a 3^b 5^c 7^d");
};

// LDS placement of element n of sequence s: one pad slot every 32 elements
// breaks the power-of-two strides of the Stockham write pattern.
template <int N> struct Lds {
    static constexpr int P = N + N / 32 + 1;           // sequence pitch
    __device__ __forceinline__ static int at(int s, int n) { return s * P + n + (n >> 5); }
};

// One Stockham stage over NSEQ sequences of length N in LDS, in place:
// task (s, j), j < N/R, reads x[j + r N/R], applies w^(r (j mod NS)) with
// w = exp(DIR 2 pi i / (NS R)), does a length-R DFT, and writes
// y[(j / NS) NS R + (j mod NS) + r NS].
template <typename T, int N, int R, int NS, int NSEQ, int NT, int DIR>
__device__ __forceinline__ void stockham_stage(C2<T>* buf, const C2<T>* tw, int tid) {
    constexpr int M = N / R;
    constexpr int TASKS = NSEQ * M;
    constexpr int TPT = (TASKS + NT - 1) / NT;
    C2<T> v[TPT][R];
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int task = tid + q * NT;
        if (TASKS % NT == 0 || task < TASKS) {
            const int s = task / M, j = task % M;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[Lds<N>::at(s, j + r * M)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
        const int task = tid + q * NT;
        if (TASKS % NT == 0 || task < TASKS) {
            const int s = task / M, j = task % M;
            const int jm = j % NS;
            if constexpr (NS > 1) {
                constexpr int STEP = N / (NS * R);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C2<T> w = tw[r * jm * STEP];
                    if (DIR > 0) w = cconj(w);
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            dftR<T, R, DIR>(v[q]);
            const int base = (j / NS) * NS * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[Lds<N>::at(s, base + r * NS)] = v[q][r];
        }
    }
    __syncthreads();
}

template <typename T, int N, int NSEQ, int NT, int DIR, int S = 0, int NS = 1>
__device__ __forceinline__ void fft_lds(C2<T>* buf, const C2<T>* tw, int tid) {
    if constexpr (S < Plan<N>::nst) {
        constexpr int R = Plan<N>::radix(S);
        stockham_stage<T, N, R, NS, NSEQ, NT, DIR>(buf, tw, tid);
        fft_lds<T, N, NSEQ, NT, DIR, S + 1, NS * R>(buf, tw, tid);
    }
}

// ---------------------------------------------------------------------------
// Lane-group FFT.  A transform of length N is held by G = N / E consecutive
// threads ("lanes" u = 0..G-1), E elements each, in the cyclic layout
// x[e] = data[u + G e].  Every Stockham stage reads this layout (constant
// geometry), so stage inputs come straight from registers; outputs are
// exchanged through an LDS region of the group, except after the last stage,
// whose outputs land back in the cyclic layout in registers.  Radices must
// divide E (each lane then runs E / R butterflies per stage).
template <int N, int E> struct LGPlan {
    static constexpr int a = log2_part(N);
    static constexpr int b = log3_part(N);
    static constexpr int c5 = logp_part(N, 5);
    static constexpr int c7 = logp_part(N, 7);
    static constexpr int ea = log2_part(E);
    // radix-8 stages if 8 | E, then 4s (if 4 | E) and 2s, then radix-3, 5, 7
    static constexpr int r8 = (ea >= 3) ? a / 3 : 0;
    static constexpr int rest = a - 3 * r8;              // remaining power of two
    static constexpr int n4 = (ea >= 2) ? rest / 2 : 0;
    static constexpr int n2 = rest - 2 * n4;
    static constexpr int p2 = r8 + n4 + n2;
    static constexpr int nst = p2 + b + c5 + c7;
    static constexpr int radix(int s) {
        return s < r8 ? 8 : (s < r8 + n4 ? 4 : (s < p2 ? 2 : (s < p2 + b ? 3 : (s < p2 + b + c5 ? 5 : 7))));
    }
    static_assert(b == 0 || E % 3 == 0, "radix-3 stages need 3 | E");
    static_assert(c5 == 0 || E % 5 == 0, "radix-5 stages need 5 | E");
    static_assert(c7 == 0 || E % 7 == 0, "radix-7 stages need 7 | E");
    static_assert(N % E == 0 && (N / E) <= 1024, "bad lane-group shape");
};

// Element n of a lane-group's LDS region sits at base[n * S + pad(n)]:
// S2 = 1 adds one pad slot every 32 elements, S2 = 8 one every 8 elements
// (contiguous regions; the finer pad spreads the 8-element runs of the
// radix-8 Stockham writes over distinct banks), S2 = 0 none; S > 1
// interleaves the regions of neighbouring groups (column tiles).
template <int N, int S, int S2> struct LgAt {
    static constexpr int PSH = S2 == 8 ? 3 : 5;
    static constexpr int PAD = S2 == 8 ? 1 : S2;
    __device__ __forceinline__ static int at(int n) { return n * S + (n >> PSH) * PAD; }
    static constexpr int span = (N - 1) * S + ((N - 1) >> PSH) * PAD + 1;
};

// Orders one wave's LDS writes before its later LDS reads (a wave's LDS
// operations complete in issue order; the fences keep the compiler from
// moving memory operations across the point).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Barrier of a lane group's exchange: the whole block, or only the wave when
// every lane group lies inside one wave (WAVE).
template <bool WAVE> __device__ __forceinline__ void lg_sync() {
    if constexpr (WAVE) wave_sync();
    else __syncthreads();
}

template <typename T, int N, int E, int R, int NS, int DIR, int S, int S2, int TWN, bool WAVE = false>
__device__ __forceinline__ void lg_stage_tw(C2<T> (&x)[E], C2<T>* reg, const C2<T>* tw, int u) {
    constexpr int G = N / E, Q = E / R;
    constexpr bool LAST = (NS * R == N);
    using A = LgAt<N, S, S2>;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = u + G * q;
        C2<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[q + Q * r];
        const int jm = j % NS;
        if constexpr (NS > 1) {
            constexpr int STEP = (TWN / N) * (N / (NS * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C2<T> w = tw[r * jm * STEP];
                if (DIR > 0) w = cconj(w);
                v[r] = cmul(v[r], w);
            }
        }
        dftR<T, R, DIR>(v);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[q + Q * r] = v[r];
        } else {
            const int base = (j / NS) * NS * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) reg[A::at(base + r * NS)] = v[r];
        }
    }
    if constexpr (!LAST) {
        lg_sync<WAVE>();
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = reg[A::at(u + G * e)];
        lg_sync<WAVE>();
    }
}

// Two independent lane-group transforms of one shape whose stages share
// their barriers: both compute, both exchange through their own LDS regions
// (rega, regb must not overlap), one pair of barriers per stage.
template <typename T, int N, int E, int R, int NS, int DIR, int S, int S2, int TWN>
__device__ __forceinline__ void lg_stage_compute(C2<T> (&x)[E], C2<T>* reg, const C2<T>* tw, int u) {
    constexpr int G = N / E, Q = E / R;
    constexpr bool LAST = (NS * R == N);
    using A = LgAt<N, S, S2>;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = u + G * q;
        C2<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[q + Q * r];
        const int jm = j % NS;
        if constexpr (NS > 1) {
            constexpr int STEP = (TWN / N) * (N / (NS * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C2<T> w = tw[r * jm * STEP];
                if (DIR > 0) w = cconj(w);
                v[r] = cmul(v[r], w);
            }
        }
        dftR<T, R, DIR>(v);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[q + Q * r] = v[r];
        } else {
            const int base = (j / NS) * NS * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) reg[A::at(base + r * NS)] = v[r];
        }
    }
}

// TAIL = false drops the barrier after the last exchange's reads: for callers
// whose next LDS writes go to other regions, with a barrier between them and
// the next writes to these.
template <typename T, int N, int E, int DIR, int S, int S2, int TWN = N, int ST = 0, int NS = 1, bool TAIL = true>
__device__ __forceinline__ void lg_fft2(C2<T> (&xa)[E], C2<T> (&xb)[E], C2<T>* rega, C2<T>* regb, const C2<T>* tw,
                                        int u) {
    if constexpr (ST < LGPlan<N, E>::nst) {
        constexpr int R = LGPlan<N, E>::radix(ST);
        constexpr int G = N / E;
        using A = LgAt<N, S, S2>;
        lg_stage_compute<T, N, E, R, NS, DIR, S, S2, TWN>(xa, rega, tw, u);
        lg_stage_compute<T, N, E, R, NS, DIR, S, S2, TWN>(xb, regb, tw, u);
        if constexpr (NS * R != N) {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                xa[e] = rega[A::at(u + G * e)];
                xb[e] = regb[A::at(u + G * e)];
            }
            if constexpr (TAIL || ST + 2 < LGPlan<N, E>::nst) __syncthreads();
        }
        lg_fft2<T, N, E, DIR, S, S2, TWN, ST + 1, NS * R, TAIL>(xa, xb, rega, regb, tw, u);
    }
}

// tw: table of TWN entries exp(-2 pi i e / TWN), TWN a multiple of N.
// WAVE: every lane group lies inside one wave (N / E divides 64 and groups
// start at multiples of N / E), so exchanges only order the wave's own LDS
// accesses; the caller still synchronises the block around the transform
// wherever other lane groups touch this group's region.
template <typename T, int N, int E, int DIR, int S, int S2, int TWN = N, int ST = 0, int NS = 1, bool WAVE = false>
__device__ __forceinline__ void lg_fft(C2<T> (&x)[E], C2<T>* reg, const C2<T>* tw, int u) {
    static_assert(!WAVE || 64 % (N / E) == 0, "a wave-synchronised lane group must fit in one wave");
    if constexpr (ST < LGPlan<N, E>::nst) {
        constexpr int R = LGPlan<N, E>::radix(ST);
        lg_stage_tw<T, N, E, R, NS, DIR, S, S2, TWN, WAVE>(x, reg, tw, u);
        lg_fft<T, N, E, DIR, S, S2, TWN, ST + 1, NS * R, WAVE>(x, reg, tw, u);
    }
}

// Copy a twiddle table of N entries into LDS (caller synchronises).
template <typename T, int N, int NT>
__device__ __forceinline__ void load_twiddles(C2<T>* dst, const C2<T>* __restrict__ src, int tid) {
    for (int e = tid; e < N; e += NT) dst[e] = src[e];
}

// The same copy in two halves: fetch() requests a thread's table entries into
// registers and store() writes them to LDS, so that a kernel can request its
// data rows in between and wait for the table alone (memory requests
// complete in order) instead of for a round trip before its first row.
template <typename T, int N, int NT> struct TwiddleCopy {
    static constexpr int K = (N + NT - 1) / NT;
    C2<T> r[K];
    __device__ __forceinline__ void fetch(const C2<T>* __restrict__ src, int tid) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (tid + k * NT < N) r[k] = src[tid + k * NT];
    }
    __device__ __forceinline__ void store(C2<T>* dst, int tid) const {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (tid + k * NT < N) dst[tid + k * NT] = r[k];
    }
};

}  // namespace tf
