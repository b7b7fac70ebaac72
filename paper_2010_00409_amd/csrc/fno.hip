// Learned surrogate: a Fourier neural operator that maps eight pulse and
// optics parameters to the six-component focal-window field, trained on the
// solver's own output.  The paper motivates fast generation of many focusing
// runs as training data for learned models (Sec. I and Sec. III.B.3); the
// operator itself is this library's.
//
// Architecture (fixed): 64^3 window, width 32, 12 kept modes per axis
// (kx in [0, 12), ky and kz in [0, 12) U [52, 64)), 3 Fourier layers,
// projection 32 -> 128 -> 6, GELU(x) = x (1 + erf(x / sqrt 2)) / 2.
//   v0      = [p, x, y, z] W0 + b0                      (lift, fp32)
//   z_l     = irfft3(R_l . rfft3(v_l)|kept) + v_l W_l + b_l
//   v_l+1   = GELU(z_l) (l < 2),  v_3 = z_2
//   out     = GELU(v_3 P1 + c1) P2 + c2
// Loss: mean over samples of ||out - y|| / ||y||.
//
// Arithmetic: every contraction runs on bf16 MFMA with fp32 accumulation.
// Learned weights enter as bf16 working copies of fp32 master weights; the
// truncated DFT matrices (float64-built) and the activations they multiply
// are split into bf16 hi + lo parts and multiplied with three MFMAs, which
// keeps the spectral transforms at about fp32 accuracy.
//
// Data layout (fp32, one sample; B samples are stacked outermost):
//   node tensor  [z][y][x][c]                 64^3 x 32, channel fastest
//   X1 (x pass)  [z][y][s][kx][c]             s: 0 real, 1 imaginary
//   X2 (y pass)  [ky][z][s][kx][c]
//   modes        [kz][s][ky][kx][c]           mode q = (kz * 24 + ky) * 12 + kx
//   out, target  [6][z][y][x]
// Every stage is "a small constant matrix applied along one axis" and runs as
// one strided GEMM whose row/column index maps are two-level affine.
#include "engine.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>

namespace tf {
namespace fno {

constexpr int N = 64, N3 = N * N * N, C = 32, M = 12, NPAR = 8, HID = 128, NOUT = 6, LAYERS = 3;
constexpr int KS = 2 * M;                 // kept ky / kz values
constexpr int NMODES = KS * KS * M;       // 6912
constexpr int LINE = M * C;               // 384 floats: one (kx, c) block
constexpr int64_t NODE_SZ = int64_t(N3) * C;                // node tensor per sample
constexpr int64_t X1_SZ = int64_t(N) * N * 2 * LINE;        // 3,145,728
constexpr int64_t X2_SZ = int64_t(KS) * N * 2 * LINE;       // 1,179,648
constexpr int64_t X3_SZ = int64_t(KS) * 2 * KS * LINE;      // 442,368
constexpr int64_t OUT_SZ = int64_t(NOUT) * N3;
constexpr int CHUNK = 4096;               // nodes per split-K block of the weight gradients
constexpr int KSLOTS = 4 * 2 * 2 * 32 * 8; // one 128-row operand in kappa fragment order
constexpr int NCHUNK = N3 / CHUNK;

// Flat parameter vector (fp32): W0 (11x32), b0, then per layer W (32x32),
// b (32), R (NMODES x 32 x 32 complex as [q][c][o][re, im]), then P1 (32x128),
// c1, P2 (128 x 6K), c2 (6K) for a head of K basis fields.  Row-major, input
// index first.
constexpr int64_t OFF_W0 = 0, OFF_B0 = 11 * C;
constexpr int64_t LAYER_SZ = C * C + C + int64_t(NMODES) * C * C * 2;
constexpr int64_t OFF_L0 = OFF_B0 + C;
constexpr int64_t off_w(int l) { return OFF_L0 + l * LAYER_SZ; }
constexpr int64_t off_b(int l) { return off_w(l) + C * C; }
constexpr int64_t off_r(int l) { return off_b(l) + C; }
constexpr int64_t OFF_P1 = OFF_L0 + LAYERS * LAYER_SZ;
constexpr int64_t OFF_C1 = OFF_P1 + C * HID;
constexpr int64_t OFF_P2 = OFF_C1 + HID;
constexpr int64_t off_c2(int nb) { return OFF_P2 + int64_t(HID) * NOUT * nb; }
constexpr int64_t nparams(int nb) { return off_c2(nb) + NOUT * nb; }

typedef __bf16 bf16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// erf by Abramowitz & Stegun 7.1.28 (|error| <= 3e-7; about 2e-6 after
// float32 rounding, far below the bf16 rounding of every value a GELU
// feeds): for u >= 0, erf(u) = 1 - 1 / (1 + a1 u + ... + a6 u^6)^16.  One
// reciprocal and no exponential; large u gives an infinite power and 1.
__device__ __forceinline__ float erf_as(float u) {
    const float a = fabsf(u);
    const float q = 1.0f + a * (0.0705230784f + a * (0.0422820123f + a * (0.0092705272f +
                                a * (0.0001520143f + a * (0.0002765672f + a * 0.0000430638f)))));
    const float q2 = q * q, q4 = q2 * q2, q8 = q4 * q4;
    const float r = 1.0f - __builtin_amdgcn_rcpf(q8 * q8);
    return u < 0.0f ? -r : r;
}
__device__ __forceinline__ float gelu(float x) {
    return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f));
}
// GELU'(x) = Phi(x) + x phi(x), with the standard normal density phi
__device__ __forceinline__ float gelu_d(float x) {
    const float ex = __expf(-0.5f * x * x);
    return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) + x * ex * 0.39894228040143268f;
}

__device__ __forceinline__ float ldf(const float* p) { return *p; }
__device__ __forceinline__ float ldf(const bf16* p) { return (float)*p; }

// ---------------------------------------------------------------------------
// Generic strided GEMM  C[b] = alpha * A[b] (M x K) . B[b] (K x N)  (+= C[b])
// ---------------------------------------------------------------------------

// Two-level affine index map: i -> (i >> sh) * hi + (i & (2^sh - 1)) * lo.
struct Ix {
    int sh, hi, lo;
};
__host__ __device__ __forceinline__ int64_t ixoff(Ix a, int i) {
    return int64_t(i >> a.sh) * a.hi + int64_t(i & ((1 << a.sh) - 1)) * a.lo;
}

struct Operand {
    const void* p;        // nullptr: every element is 1
    int64_t b1, b2;       // element strides of blockIdx.y and blockIdx.z
    Ix r, c;              // row and column maps
    int ones_from;        // rows >= ones_from read 1 (A only; large value: none)
    int fast_k;           // consecutive threads walk k (k is the contiguous index)
    int vec;              // groups of 4 along the contiguous index are contiguous and aligned
};
struct Result {
    float* p;
    int64_t b1, b2;
    Ix r, c;
    float alpha;
    int accumulate;
};
struct GemmArgs {
    Operand a, b;
    Result c;
    int M, N, K;
};

__device__ __forceinline__ void ld4(const float* p, float v[4]) {
    const float4 q = *(const float4*)p;
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
__device__ __forceinline__ void ld4(const bf16* p, float v[4]) {
    const uint2 q = *(const uint2*)p;           // element 0 in the low half
    v[0] = __uint_as_float(q.x << 16); v[1] = __uint_as_float(q.x & 0xffff0000u);
    v[2] = __uint_as_float(q.y << 16); v[3] = __uint_as_float(q.y & 0xffff0000u);
}

// Stage a ROWS x 32 slice of an operand in LDS as bf16 (hi and, for SPLIT,
// lo parts), k contiguous.  "Rows" are the M index of A or the N index of B.
// Each thread owns one row and 8 consecutive k and stores them with one
// 16-byte LDS write per part.  Neighbouring threads take neighbouring k
// groups when k is the contiguous index in memory (two 16-byte global loads
// when aligned), else neighbouring rows (coalesced 4-byte loads); either way
// the 16-byte writes of a quarter-wave start 20 banks apart (row pitch 80 B)
// or are contiguous, so they do not collide.
template <int ROWS, int NT, typename TT, bool SPLIT, bool IS_B>
__device__ __forceinline__ void stage(bf16* s0, bf16* s1, const TT* P, const Operand& o, int r0, int k0, int nrows,
                                      int K) {
    constexpr int BK = 32, PITCH = BK + 8, KG = BK / 8;
    auto off = [&](int gr, int gk) -> int64_t {
        return IS_B ? ixoff(o.r, gk) + ixoff(o.c, gr) : ixoff(o.r, gr) + ixoff(o.c, gk);
    };
    for (int t = threadIdx.x; t < ROWS * KG; t += NT) {
        int rr, kg;
        if (o.fast_k) { rr = t / KG; kg = t % KG; }
        else          { rr = t % ROWS; kg = t / ROWS; }
        const int gr = r0 + rr, gk0 = k0 + 8 * kg;
        float v[8];
        if (gr >= nrows) {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = 0.0f;
        } else if (!P || (!IS_B && gr >= o.ones_from)) {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = gk0 + e < K ? 1.0f : 0.0f;
        } else if (o.vec && o.fast_k && gk0 + 8 <= K) {
            ld4(P + off(gr, gk0), v);
            ld4(P + off(gr, gk0 + 4), v + 4);
        } else if (gk0 + 8 <= K) {
            const int64_t orow = IS_B ? ixoff(o.c, gr) : ixoff(o.r, gr);
            const Ix kmap = IS_B ? o.r : o.c;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = ldf(P + orow + ixoff(kmap, gk0 + e));
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = gk0 + e < K ? ldf(P + off(gr, gk0 + e)) : 0.0f;
        }
        bf16x8 hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const bf16 h = (bf16)v[e];
            hi[e] = h;
            lo[e] = (bf16)(v[e] - (float)h);
        }
        *(bf16x8*)&s0[rr * PITCH + 8 * kg] = hi;
        if constexpr (SPLIT) *(bf16x8*)&s1[rr * PITCH + 8 * kg] = lo;
    }
}

// Each wave owns 32x32 output sub-tiles; the K loop stages 32-wide slices of
// A and B in LDS as bf16 (hi and, for SPLIT, lo parts), k contiguous so each
// lane reads its eight k values with one 16-byte LDS load.
template <int BM, int BN, int NW, typename TA, typename TB, bool SPLIT>
__global__ __launch_bounds__(64 * NW) void k_gemm(GemmArgs g) {
    constexpr int BK = 32, PITCH = BK + 8, NT = 64 * NW;
    constexpr int SUBN = BN / 32, SUB = (BM / 32) * SUBN, PER = SUB / NW;
    static_assert(SUB % NW == 0, "sub-tiles must divide among the waves");
    constexpr int NP = SPLIT ? 2 : 1;
    __shared__ __attribute__((aligned(16))) bf16 sa[NP][BM * PITCH];
    __shared__ __attribute__((aligned(16))) bf16 sb[NP][BN * PITCH];

    const int tilesN = (g.N + BN - 1) / BN;
    const int m0 = (blockIdx.x / tilesN) * BM, n0 = (blockIdx.x % tilesN) * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = lane & 31, grp = lane >> 5;
    const TA* A = g.a.p ? (const TA*)g.a.p + blockIdx.y * g.a.b1 + blockIdx.z * g.a.b2 : nullptr;
    const TB* B = g.b.p ? (const TB*)g.b.p + blockIdx.y * g.b.b1 + blockIdx.z * g.b.b2 : nullptr;

    f32x16 acc[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[p][r] = 0.0f;

    for (int k0 = 0; k0 < g.K; k0 += BK) {
        stage<BM, NT, TA, SPLIT, false>(sa[0], sa[NP - 1], A, g.a, m0, k0, g.M, g.K);
        stage<BN, NT, TB, SPLIT, true>(sb[0], sb[NP - 1], B, g.b, n0, k0, g.N, g.K);
    __syncthreads();
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int st = wave * PER + p, mt = st / SUBN, nt = st % SUBN;
#pragma unroll
            for (int ks = 0; ks < BK / 16; ++ks) {
                const int ao = (mt * 32 + t) * PITCH + ks * 16 + 8 * grp;
                const int bo = (nt * 32 + t) * PITCH + ks * 16 + 8 * grp;
                const bf16x8 ah = *(const bf16x8*)&sa[0][ao];
                const bf16x8 bh = *(const bf16x8*)&sb[0][bo];
                acc[p] = mfma(ah, bh, acc[p]);
                if constexpr (SPLIT) {
                    const bf16x8 al = *(const bf16x8*)&sa[NP - 1][ao];
                    const bf16x8 bl = *(const bf16x8*)&sb[NP - 1][bo];
                    acc[p] = mfma(ah, bl, acc[p]);
                    acc[p] = mfma(al, bh, acc[p]);
                }
            }
        }
        __syncthreads();
    }

    float* Cp = g.c.p + blockIdx.y * g.c.b1 + blockIdx.z * g.c.b2;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int st = wave * PER + p, mt = st / SUBN, nt = st % SUBN;
        const int col = n0 + nt * 32 + t;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = m0 + mt * 32 + 8 * (r >> 2) + 4 * grp + (r & 3);
            if (row < g.M && col < g.N) {
                float* d = Cp + ixoff(g.c.r, row) + ixoff(g.c.c, col);
                const float v = g.c.alpha * acc[p][r];
                *d = g.c.accumulate ? *d + v : v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Fused per-line kernels
// ---------------------------------------------------------------------------

// One wave per x-line (64 nodes, two 32-node halves):
//   acc[x][j] = sum_k CM[x][k] LN[k][j]   (k < 24, split bf16)
//             + sum_c ACT[x][c] Wt[c][j]  (bf16)
// Forward (inverse x transform + pointwise branch of a layer):
//   CM = inverse x matrix, LN = the line's (s, kx) x c block, Wt = W,
//   z = acc + b; zout <- z; out <- GELU(z) or z.
// Backward (adjoint): CM = transpose of the forward x matrix, LN = gradient
//   block, ACT = dL/dz_l, Wt = W^T; out <- acc * GELU'(z_{l-1}) or acc.
struct LineArgs {
    const float* cm;      // [64][24]
    const float* ln;      // [lines][24][32]
    const float* act;     // [lines][64][32], or nullptr: no pointwise term
    const bf16* w;        // [32][32] row-major W[c][o]
    const float* bias;    // [32] (forward) or nullptr
    const float* zprev;   // backward: z_{l-1} for GELU', or nullptr
    float* zout;          // forward: pre-activation, or nullptr
    float* out;
    int nlines;
    int bwd;
    int act_gelu;         // forward: out = GELU(z)
};

__global__ __launch_bounds__(256) void k_lineout(LineArgs a) {
    const int lane = threadIdx.x & 63, t = lane & 31, grp = lane >> 5;
    const int line = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (line >= a.nlines) return;

    // constant fragments: CM rows (split) and the weight columns
    bf16x8 cmh[2][2], cml[2][2], wf[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 16 * s + 8 * grp + e;
                const float v = k < 24 ? a.cm[(32 * h + t) * 24 + k] : 0.0f;
                const bf16 hi = (bf16)v;
                cmh[h][s][e] = hi;
                cml[h][s][e] = (bf16)(v - (float)hi);
            }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 16 * s + 8 * grp + e;
            wf[s][e] = a.bwd ? a.w[t * C + k] : a.w[k * C + t];
        }

    // spectral block of this line as the B operand (k = (s, kx) < 24, column t)
    const float* ln = a.ln + int64_t(line) * 24 * C;
    bf16x8 lh[2], ll[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 16 * s + 8 * grp + e;
            const float v = k < 24 ? ln[k * C + t] : 0.0f;
            const bf16 hi = (bf16)v;
            lh[s][e] = hi;
            ll[s][e] = (bf16)(v - (float)hi);
        }

    const int64_t base = int64_t(line) * N * C;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            acc = mfma(cmh[h][s], lh[s], acc);
            acc = mfma(cmh[h][s], ll[s], acc);
            acc = mfma(cml[h][s], lh[s], acc);
        }
        if (a.act) {
            const float* ap = a.act + base + (32 * h + t) * C + 8 * grp;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const float4 u0 = *(const float4*)(ap + 16 * s);
                const float4 u1 = *(const float4*)(ap + 16 * s + 4);
                bf16x8 af;
                af[0] = (bf16)u0.x; af[1] = (bf16)u0.y; af[2] = (bf16)u0.z; af[3] = (bf16)u0.w;
                af[4] = (bf16)u1.x; af[5] = (bf16)u1.y; af[6] = (bf16)u1.z; af[7] = (bf16)u1.w;
                acc = mfma(af, wf[s], acc);
            }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int x = 32 * h + 8 * (r >> 2) + 4 * grp + (r & 3);
            const int64_t idx = base + x * C + t;
            float v = acc[r];
            if (!a.bwd) {
                if (a.bias) v += a.bias[t];
                if (a.zout) a.zout[idx] = v;
                a.out[idx] = a.act_gelu ? gelu(v) : v;
            } else {
                if (a.zprev) v *= gelu_d(a.zprev[idx]);
                a.out[idx] = v;
            }
        }
    }
}

// Projection 32 -> 128 -> 6 per 32-node tile, one wave per tile.  The hidden
// layer is computed transposed (h^T = P1^T v^T): its MFMA accumulator holds,
// in lane (node t, group g), register r, the hidden unit
//   kappa(r) = 8 (r >> 2) + 4 g + (r & 3)  within a 32-unit block,
// which is exactly the k slot an MFMA operand in that lane needs when the
// K index is relabelled by kappa.  So the hidden layer feeds the next
// contraction straight from registers, with the constant operand (P2 or P1)
// gathered in the same kappa order.
struct ProjArgs {
    const float* v;       // [B][N3][32]
    const bf16* p1;       // [32][128]
    const float* c1;      // [128]
    const bf16* p2;       // [B][128][6]: the head's effective projection per sample
    const float* c2;      // [B][6]
    float* out;           // forward: [B][6][N3]
    const float* gout;    // backward: dL/dout [B][6][N3]
    float* gv;            // backward: [B][N3][32]
    bf16* hT;             // backward: GELU(hidden) [B][128][N3]
    bf16* ghT;            // backward: dL/d(pre-activation) [B][128][N3]
    int ntiles;
    int bwd;
};

__device__ __forceinline__ int kappa(int s, int grp, int e) { return 16 * s + 8 * (e >> 2) + 4 * grp + (e & 3); }

__global__ __launch_bounds__(256) void k_proj(ProjArgs a) {
    const int lane = threadIdx.x & 63, t = lane & 31, grp = lane >> 5;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;
    const int b = tile / (N3 / 32), node0 = (tile % (N3 / 32)) * 32;

    // A operand of h^T = P1^T v^T: lane (hidden 32 mt + t), k = c
    bf16x8 p1t[4][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) p1t[mt][s][e] = a.p1[(16 * s + 8 * grp + e) * HID + 32 * mt + t];

    // B operand v^T: lane (node t), k = c
    bf16x8 vf[2];
    {
        const float* vp = a.v + (int64_t(b) * N3 + node0 + t) * C + 8 * grp;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float4 u0 = *(const float4*)(vp + 16 * s);
            const float4 u1 = *(const float4*)(vp + 16 * s + 4);
            vf[s][0] = (bf16)u0.x; vf[s][1] = (bf16)u0.y; vf[s][2] = (bf16)u0.z; vf[s][3] = (bf16)u0.w;
            vf[s][4] = (bf16)u1.x; vf[s][5] = (bf16)u1.y; vf[s][6] = (bf16)u1.z; vf[s][7] = (bf16)u1.w;
        }
    }

    const bf16* p2 = a.p2 + int64_t(b) * HID * NOUT;
    const float* c2 = a.c2 + b * NOUT;
    if (!a.bwd) {
        f32x16 oacc;
#pragma unroll
        for (int r = 0; r < 16; ++r) oacc[r] = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
            acc = mfma(p1t[mt][0], vf[0], acc);
            acc = mfma(p1t[mt][1], vf[1], acc);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                bf16x8 hf, pf;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int hd = 32 * mt + kappa(s, grp, e);
                    hf[e] = (bf16)gelu(acc[8 * s + e] + a.c1[hd]);
                    pf[e] = t < NOUT ? p2[hd * NOUT + t] : (bf16)0.0f;
                }
                oacc = mfma(pf, hf, oacc);
            }
        }
        // rows are output components: group 0 holds 0..3 (r = 0..3), group 1 holds 4, 5 (r = 0, 1)
        float* op = a.out + int64_t(b) * OUT_SZ + node0 + t;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * grp + r;
            if (o < NOUT) op[int64_t(o) * N3] = oacc[r] + c2[o];
        }
        return;
    }

    // backward: dL/dout^T as the B operand of dL/dh^T = P2 . dL/dout^T (K = 6 padded to 16)
    bf16x8 gf;
    {
        const float* gp = a.gout + int64_t(b) * OUT_SZ + node0 + t;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int o = 8 * grp + e;
            gf[e] = o < NOUT ? (bf16)gp[int64_t(o) * N3] : (bf16)0.0f;
        }
    }
    f32x16 gvacc;
#pragma unroll
    for (int r = 0; r < 16; ++r) gvacc[r] = 0.0f;
    bf16* hp = a.hT + int64_t(b) * HID * N3 + node0 + t;
    bf16* ghp = a.ghT + int64_t(b) * HID * N3 + node0 + t;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x16 acc, gacc;
#pragma unroll
        for (int r = 0; r < 16; ++r) { acc[r] = 0.0f; gacc[r] = 0.0f; }
        acc = mfma(p1t[mt][0], vf[0], acc);
        acc = mfma(p1t[mt][1], vf[1], acc);
        bf16x8 p2f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int o = 8 * grp + e;
            p2f[e] = o < NOUT ? p2[(32 * mt + t) * NOUT + o] : (bf16)0.0f;
        }
        gacc = mfma(p2f, gf, gacc);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8 af, bfr;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = 8 * s + e;
                const int hd = 32 * mt + kappa(s, grp, e);
                const float pre = acc[r] + a.c1[hd];
                const float gpre = gacc[r] * gelu_d(pre);
                hp[int64_t(hd) * N3] = (bf16)gelu(pre);
                const bf16 gb = (bf16)gpre;
                ghp[int64_t(hd) * N3] = gb;
                af[e] = gb;
                bfr[e] = a.p1[t * HID + hd];
            }
            gvacc = mfma(af, bfr, gvacc);
        }
    }
    float* gvp = a.gv + (int64_t(b) * N3 + node0) * C + t;
#pragma unroll
    for (int r = 0; r < 16; ++r) gvp[(8 * (r >> 2) + 4 * grp + (r & 3)) * C] = gvacc[r];
}

// ---------------------------------------------------------------------------
// Elementwise and reduction kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ float coord(int i) { return float(i - N / 2) / float(N / 2); }

// v0[b][node][c] = b0[c] + sum_i p[b][i] W0[i][c] + x W0[8][c] + y W0[9][c] + z W0[10][c],
// always summed in this order
__device__ __forceinline__ float lift_base(const float* pb, const float* w0, const float* b0, int c) {
    float s = b0[c];
    for (int i = 0; i < NPAR; ++i) s += pb[i] * w0[i * C + c];
    return s;
}
__device__ __forceinline__ float lift_at(float base, const float* w0, int c, int x, int y, int z) {
    float s = base;
    s += coord(x) * w0[8 * C + c];
    s += coord(y) * w0[9 * C + c];
    s += coord(z) * w0[10 * C + c];
    return s;
}

__global__ void k_lift(const float* p, const float* w0, const float* b0, float* v, int64_t total) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int c = idx & (C - 1);
    const int64_t nb = idx >> 5;
    const int node = int(nb % N3), b = int(nb / N3);
    v[idx] = lift_at(lift_base(p + b * NPAR, w0, b0, c), w0, c, node % N, (node / N) % N, node / (N * N));
}

// ---------------------------------------------------------------------------
// Fused inference kernels: no activation of the forward pass is kept, and
// the first x contraction of every layer is taken from the registers of the
// kernel that produced the layer's input.
// ---------------------------------------------------------------------------

// 8 (or 4) consecutive floats from a 16-byte aligned address, or zeros
__device__ __forceinline__ void ld8(const float* p, bool in, float v[8]) {
    if (in) {
        const float4 q0 = *(const float4*)p, q1 = *(const float4*)(p + 4);
        v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w; v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.0f;
    }
}
__device__ __forceinline__ void ld4c(const float* p, bool in, float v[4]) {
    if (in) {
        const float4 q = *(const float4*)p;
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
        v[0] = v[1] = v[2] = v[3] = 0.0f;
    }
}

// element e of (hi, lo) <- bf16 split of v
__device__ __forceinline__ void split(float v, bf16x8& hi, bf16x8& lo, int e) {
    const bf16 h = (bf16)v;
    hi[e] = h;
    lo[e] = (bf16)(v - (float)h);
}

struct InfArgs {
    const float* gx;      // inverse x matrix [64][24]
    const float* fx;      // forward x matrix [24][64]
    const float* ln;      // spectral lines [lines][24][32] (U1); overwritten by the next layer's X1
    const float* act;     // v_l [lines][64][32], or nullptr: v_0 recomputed from the lift
    const float* p;       // [B][8] parameters (lift)
    const float* w0;
    const float* b0;
    const bf16* w;        // W_l [32][32]
    const float* bias;    // b_l
    float* vout;          // v_{l+1} (not the last layer)
    float* x1out;         // X1 of layer l+1, written over the line's U1
    // projection (last layer), operands in kappa fragment order
    const bf16* p1k;      // [4][2][2][32][8]
    const float* c1;
    const bf16* p2k;      // [B][4][2][2][32][8]
    const float* c2e;     // [B][6]
    float* out;           // [B][6][N3]
    int nlines;
};

// Lift and the first x contraction, one wave per x-line:
//   X1[(s,kx)][c] = sum_x Fx[(s,kx)][x] v0[x][c]    (split bf16)
__global__ __launch_bounds__(256) void k_lift_x(InfArgs a) {
    const int lane = threadIdx.x & 63, t = lane & 31, grp = lane >> 5;
    const int line = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (line >= a.nlines) return;
    const int b = line / (N * N), zy = line % (N * N);
    const float base = lift_base(a.p + b * NPAR, a.w0, a.b0, t);
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        bf16x8 ah, al, bh, bl;
        float fr[8];
        ld8(a.fx + t * N + 16 * ks + 8 * grp, t < 24, fr);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int x = 16 * ks + 8 * grp + e;
            split(fr[e], ah, al, e);
            split(lift_at(base, a.w0, t, x, zy % N, zy / N), bh, bl, e);
        }
        acc = mfma(ah, bh, acc);
        acc = mfma(ah, bl, acc);
        acc = mfma(al, bh, acc);
    }
    float* o = a.x1out + int64_t(line) * 24 * C + t;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r >> 2) + 4 * grp + (r & 3);
        if (i < 24) o[i * C] = acc[r];
    }
}

// Inverse x transform + pointwise branch + GELU of a layer that is not the
// last, then the next layer's x contraction from the registers:
//   v[x][o]  = GELU(sum_k Gx[x][k] U1[k][o] + sum_c v_l[x][c] W[c][o] + b[o])
//   X1[i][o] = sum_x Fx[i][x] v[x][o]
// The accumulator of v holds row x = 32 h + kappa(s, g, e) in register 8 s + e
// of lane (o, g), so it is the B operand of the contraction over x with the
// constant Fx gathered in that order.
__global__ __launch_bounds__(256) void k_line_fwd(InfArgs a) {
    const int lane = threadIdx.x & 63, t = lane & 31, grp = lane >> 5;
    const int line = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (line >= a.nlines) return;
    const int b = line / (N * N), zy = line % (N * N);
    bf16x8 cmh[2][2], cml[2][2], wf[2], lh[2], ll[2];
    const float* ln = a.ln + int64_t(line) * 24 * C;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const bool in = 16 * s + 8 * grp < 24;
        float g0[8], g1[8];
        ld8(a.gx + t * 24 + 16 * s + 8 * grp, in, g0);
        ld8(a.gx + (32 + t) * 24 + 16 * s + 8 * grp, in, g1);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 16 * s + 8 * grp + e;
            wf[s][e] = a.w[k * C + t];
            split(in ? ln[k * C + t] : 0.0f, lh[s], ll[s], e);
            split(g0[e], cmh[0][s], cml[0][s], e);
            split(g1[e], cmh[1][s], cml[1][s], e);
        }
    }
    const int64_t base = int64_t(line) * N * C;
    float lb[2][8];
    if (!a.act) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) lb[s][e] = lift_base(a.p + b * NPAR, a.w0, a.b0, 16 * s + 8 * grp + e);
    }
    f32x16 acc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[h][r] = 0.0f;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            acc[h] = mfma(cmh[h][s], lh[s], acc[h]);
            acc[h] = mfma(cmh[h][s], ll[s], acc[h]);
            acc[h] = mfma(cml[h][s], lh[s], acc[h]);
        }
        const int x = 32 * h + t;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8 af;
            if (a.act) {
                const float* ap = a.act + base + x * C + 16 * s + 8 * grp;
                const float4 u0 = *(const float4*)ap;
                const float4 u1 = *(const float4*)(ap + 4);
                af[0] = (bf16)u0.x; af[1] = (bf16)u0.y; af[2] = (bf16)u0.z; af[3] = (bf16)u0.w;
                af[4] = (bf16)u1.x; af[5] = (bf16)u1.y; af[6] = (bf16)u1.z; af[7] = (bf16)u1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    af[e] = (bf16)lift_at(lb[s][e], a.w0, 16 * s + 8 * grp + e, x, zy % N, zy / N);
            }
            acc[h] = mfma(af, wf[s], acc[h]);
        }
        const float bt = a.bias[t];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int xr = 32 * h + 8 * (r >> 2) + 4 * grp + (r & 3);
            const float v = gelu(acc[h][r] + bt);
            acc[h][r] = v;
            a.vout[base + xr * C + t] = v;
        }
    }
    f32x16 xacc;
#pragma unroll
    for (int r = 0; r < 16; ++r) xacc[r] = 0.0f;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8 ah, al, bh, bl;
            // kappa(s, g, e) for e = 0..3 and 4..7 is two runs of 4 consecutive x
            float fr[8];
            ld4c(a.fx + t * N + 32 * h + 16 * s + 4 * grp, t < 24, fr);
            ld4c(a.fx + t * N + 32 * h + 16 * s + 8 + 4 * grp, t < 24, fr + 4);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                split(fr[e], ah, al, e);
                split(acc[h][8 * s + e], bh, bl, e);
            }
            xacc = mfma(ah, bh, xacc);
            xacc = mfma(ah, bl, xacc);
            xacc = mfma(al, bh, xacc);
        }
    float* o = a.x1out + int64_t(line) * 24 * C + t;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r >> 2) + 4 * grp + (r & 3);
        if (i < 24) o[i * C] = xacc[r];
    }
}

// Last layer fused with the projection.  The layer is computed transposed,
// v^T[o][x] = sum_k U1^T[o][k] Gx^T[k][x] + sum_c W^T[o][c] v_l^T[c][x] + b[o],
// so lane (x, g) holds channel o = kappa(s, g, e) in register 8 s + e: the B
// operand of h^T = P1^T v^T over c, with P1 gathered in that order.  The
// projection then runs as in k_proj.
__global__ __launch_bounds__(256) void k_line_proj(InfArgs a) {
    const int lane = threadIdx.x & 63, t = lane & 31, grp = lane >> 5;
    // one wave per half line (32 nodes): twice the independent waves
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int line = item >> 1, h = item & 1;
    if (line >= a.nlines) return;
    const int b = line / (N * N), zy = line % (N * N);
    bf16x8 wf[2], lh[2], ll[2];
    const float* ln = a.ln + int64_t(line) * 24 * C;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 16 * s + 8 * grp + e;
            wf[s][e] = a.w[k * C + t];
            split(k < 24 ? ln[k * C + t] : 0.0f, lh[s], ll[s], e);
        }
    const bf16x8* p1k = (const bf16x8*)a.p1k + grp * 32 + t;          // + (mt * 2 + s) * 64
    const bf16x8* p2k = (const bf16x8*)(a.p2k + int64_t(b) * KSLOTS) + grp * 32 + t;
    const float* c2 = a.c2e + b * NOUT;
    const int64_t base = int64_t(line) * N * C;
    {
        const int x = 32 * h + t;
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8 cmh, cml;
            float gr[8];
            ld8(a.gx + x * 24 + 16 * s + 8 * grp, 16 * s + 8 * grp < 24, gr);
#pragma unroll
            for (int e = 0; e < 8; ++e) split(gr[e], cmh, cml, e);
            acc = mfma(lh[s], cmh, acc);
            acc = mfma(ll[s], cmh, acc);
            acc = mfma(lh[s], cml, acc);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float* ap = a.act + base + x * C + 16 * s + 8 * grp;
            const float4 u0 = *(const float4*)ap;
            const float4 u1 = *(const float4*)(ap + 4);
            bf16x8 af;
            af[0] = (bf16)u0.x; af[1] = (bf16)u0.y; af[2] = (bf16)u0.z; af[3] = (bf16)u0.w;
            af[4] = (bf16)u1.x; af[5] = (bf16)u1.y; af[6] = (bf16)u1.z; af[7] = (bf16)u1.w;
            acc = mfma(wf[s], af, acc);
        }
        bf16x8 vf[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) vf[s][e] = (bf16)(acc[8 * s + e] + a.bias[kappa(s, grp, e)]);
        f32x16 oacc;
#pragma unroll
        for (int r = 0; r < 16; ++r) oacc[r] = 0.0f;
#pragma unroll 1
        for (int mt = 0; mt < 4; ++mt) {
            f32x16 hacc;
#pragma unroll
            for (int r = 0; r < 16; ++r) hacc[r] = 0.0f;
#pragma unroll
            for (int s = 0; s < 2; ++s) hacc = mfma(p1k[(mt * 2 + s) * 64], vf[s], hacc);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                bf16x8 hf;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int hd = 32 * mt + kappa(s, grp, e);
                    hf[e] = (bf16)gelu(hacc[8 * s + e] + a.c1[hd]);
                }
                oacc = mfma(p2k[(mt * 2 + s) * 64], hf, oacc);
            }
        }
        float* op = a.out + int64_t(b) * OUT_SZ + int64_t(zy) * N + x;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * grp + r;
            if (o < NOUT) op[int64_t(o) * N3] = oacc[r] + c2[o];
        }
    }
}

// per (sample, z plane): sum_node g, and sum_node coord_d g, for every channel
__global__ __launch_bounds__(256) void k_lift_grad_part(const float* gv, float* part) {
    const int z = blockIdx.x, b = blockIdx.y;
    const int c = threadIdx.x & 31, ng = threadIdx.x >> 5;
    const float* g = gv + (int64_t(b) * N3 + int64_t(z) * N * N) * C;
    float s = 0, sx = 0, sy = 0;
    for (int nd = ng; nd < N * N; nd += 8) {
        const float v = g[nd * C + c];
        s += v;
        sx += coord(nd % N) * v;
        sy += coord(nd / N) * v;
    }
    __shared__ float red[3][8][32];
    red[0][ng][c] = s; red[1][ng][c] = sx; red[2][ng][c] = sy;
    __syncthreads();
    if (ng == 0) {
        float a0 = 0, a1 = 0, a2 = 0;
        for (int k = 0; k < 8; ++k) { a0 += red[0][k][c]; a1 += red[1][k][c]; a2 += red[2][k][c]; }
        float* o = part + (int64_t(b) * N + z) * 4 * C;
        o[c] = a0; o[C + c] = a1; o[2 * C + c] = a2; o[3 * C + c] = coord(z) * a0;
    }
}

// dL/dW0, dL/db0 from the per-plane sums (one thread per channel)
// One block of LIFT_THREADS: thread (bq, c) takes the samples b = bq (mod
// 32) in increasing b; the 32 lane sums of each of the 12 outputs are then
// added in order bq = 0..31.
constexpr int LIFT_THREADS = 1024;
__global__ __launch_bounds__(LIFT_THREADS) void k_lift_grad_final(const float* part, const float* p, int B,
                                                                  float* grad) {
    constexpr int NQ = LIFT_THREADS / C, NV = 12;
    const int c = threadIdx.x % C, bq = threadIdx.x / C;
    float gw[NV] = {0};                       // 8 parameter weights, 3 coordinate weights, bias
    for (int b = bq; b < B; b += NQ) {
        float s = 0, sx = 0, sy = 0, sz = 0;
#pragma unroll 8
        for (int z = 0; z < N; ++z) {
            const float* o = part + (int64_t(b) * N + z) * 4 * C;
            s += o[c]; sx += o[C + c]; sy += o[2 * C + c]; sz += o[3 * C + c];
        }
        for (int i = 0; i < NPAR; ++i) gw[i] += p[b * NPAR + i] * s;
        gw[8] += sx; gw[9] += sy; gw[10] += sz;
        gw[11] += s;
    }
    __shared__ float red[NQ][NV][C];
    for (int i = 0; i < NV; ++i) red[bq][i][c] = gw[i];
    __syncthreads();
    for (int idx = threadIdx.x; idx < NV * C; idx += LIFT_THREADS) {
        const int i = idx / C, cc = idx % C;
        float t = 0;
        for (int q = 0; q < NQ; ++q) t += red[q][i][cc];
        if (i < 11) grad[OFF_W0 + i * C + cc] = t;
        else grad[OFF_B0 + cc] = t;
    }
}

// per (chunk, sample): sum (out - y)^2 and sum y^2 in float64
__global__ __launch_bounds__(256) void k_loss_part(const float* out, const float* y, double* part) {
    const int ch = blockIdx.x, b = blockIdx.y;
    const int64_t len = OUT_SZ / gridDim.x;
    const float* o = out + int64_t(b) * OUT_SZ + ch * len;
    const float* t = y + int64_t(b) * OUT_SZ + ch * len;
    double sd = 0, sy = 0;
    for (int64_t i = threadIdx.x; i < len; i += 256) {
        const double d = double(o[i]) - double(t[i]);
        sd += d * d;
        sy += double(t[i]) * double(t[i]);
    }
    __shared__ double rd[256], ry[256];
    rd[threadIdx.x] = sd; ry[threadIdx.x] = sy;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) { rd[threadIdx.x] += rd[threadIdx.x + w]; ry[threadIdx.x] += ry[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[(int64_t(b) * gridDim.x + ch) * 2] = rd[0];
        part[(int64_t(b) * gridDim.x + ch) * 2 + 1] = ry[0];
    }
}

// res[0] = loss; res[1 + b] = dL/dout scale 1 / (B ||d_b|| ||y_b||).  One
// thread per sample (strided over the block); the loss sums the samples in
// order b = 0..B-1.  Launched with one block of LOSS_THREADS threads.
constexpr int LOSS_THREADS = 256;
__global__ __launch_bounds__(LOSS_THREADS) void k_loss_final(const double* part, int nch, int B, double* res,
                                                             double* ratio) {
    for (int b = threadIdx.x; b < B; b += LOSS_THREADS) {
        double sd = 0, sy = 0;
        for (int k = 0; k < nch; ++k) { sd += part[(b * nch + k) * 2]; sy += part[(b * nch + k) * 2 + 1]; }
        const double nd = sqrt(sd), ny = sqrt(sy);
        ratio[b] = nd / ny;
        res[1 + b] = nd > 0 ? 1.0 / (double(B) * nd * ny) : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double L = 0;
        for (int b = 0; b < B; ++b) L += ratio[b];
        res[0] = L / B;
    }
}

__global__ void k_gout(const float* out, const float* y, const double* res, float* g, int64_t total) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int b = int(i / OUT_SZ);
    g[i] = float(double(out[i] - y[i]) * res[1 + b]);
}

// dst[y][e] = sum_p part[y][p][e] (y = blockIdx.y), in a fixed order: a
// block takes 64 consecutive e; lane q = threadIdx.x / 64 of column e sums
// the partials p = q (mod 4) in increasing p, eight loads in flight, and
// the four lane sums are added in order q = 0..3.
__global__ __launch_bounds__(256) void k_reduce(const float* part, int nparts, int len, float* dst) {
    const int el = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + el;
    const float* src = part + int64_t(blockIdx.y) * nparts * len;
    float s = 0;
    if (e < len) {
        int p = q;
        for (; p + 28 < nparts; p += 32) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = src[int64_t(p + 4 * k) * len + e];
#pragma unroll
            for (int k = 0; k < 8; ++k) s += v[k];
        }
        for (; p < nparts; p += 4) s += src[int64_t(p) * len + e];
    }
    __shared__ float red[4][64];
    red[q][el] = s;
    __syncthreads();
    if (q == 0 && e < len)
        dst[int64_t(blockIdx.y) * len + e] = ((red[0][el] + red[1][el]) + red[2][el]) + red[3][el];
}

// dL/dR from the real 64x64 block gradient G* of Y* = X* R*:
//   re = G*[c][o] + G*[32+c][32+o],  im = G*[c][32+o] - G*[32+c][o]
__global__ void k_fold_r(const float* gs, float* gr) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(NMODES) * C * C) return;
    const int o = i & 31, c = (i >> 5) & 31;
    const float* G = gs + (i >> 10) * 4096;
    gr[2 * i] = G[c * 64 + o] + G[(32 + c) * 64 + 32 + o];
    gr[2 * i + 1] = G[c * 64 + 32 + o] - G[(32 + c) * 64 + o];
}

// bf16 working copy of R as the real block matrix R*[(s,c)][(s',o)]:
//   s = s': re,  s = 0, s' = 1: im,  s = 1, s' = 0: -im
__global__ void k_expand_r(const float* r, bf16* rb) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(NMODES) * 4096) return;
    const int j = i & 63, k = (i >> 6) & 63;
    const int64_t q = i >> 12;
    const int s = k >> 5, c = k & 31, s2 = j >> 5, o = j & 31;
    const float* e = r + ((q * C + c) * C + o) * 2;
    const float v = s == s2 ? e[0] : (s == 0 ? e[1] : -e[1]);
    rb[i] = (bf16)v;
}

// Effective projection of sample b for a head of nb basis fields:
//   P2eff[b][hd][c] = sum_k w[b][k] P2[hd][6k + c],  c2eff[b][c] = sum_k w[b][k] c2[6k + c]
// (w = 1 when nb = 1 and no weights are given).
// and in the projection's kappa order, padded to 32 outputs:
//   p2k[b][mt][s][g][t][e] = P2eff[b][32 mt + kappa(s, g, e)][t]  (0 for t >= 6)
__global__ void k_head_eff(const float* p2, const float* c2, const float* w, int nb, int B, bf16* p2e, float* c2e,
                           bf16* p2k) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = (HID + 1) * NOUT;
    if (i >= B * per) return;
    const int b = i / per, r = (i % per) / NOUT, c = i % NOUT;
    const float* src = r < HID ? p2 + int64_t(r) * NOUT * nb : c2;
    float s = 0.0f;
    for (int k = 0; k < nb; ++k) s += (w ? w[b * nb + k] : 1.0f) * src[NOUT * k + c];
    if (r < HID) {
        p2e[(int64_t(b) * HID + r) * NOUT + c] = (bf16)s;
        // r = 32 mt + kappa(s', g, e): invert kappa (16 s' + 8 (e >> 2) + 4 g + (e & 3))
        const int mt = r >> 5, q = r & 31, sp = q >> 4, eh = (q >> 3) & 1, g = (q >> 2) & 1, el = q & 3;
        const int e = 4 * eh + el;
        bf16* d = p2k + int64_t(b) * KSLOTS;
        d[((((mt * 2 + sp) * 2 + g) * 32 + c) * 8) + e] = (bf16)s;
    } else {
        c2e[b * NOUT + c] = s;
    }
}

// dL/dP2 and dL/dc2 from the per-sample gradients of the effective head
// (geff [B][129][6], row 128 the bias):  G[r][6k + c] = sum_b w[b][k] geff[b][r][c]
__global__ void k_head_grad(const float* geff, const float* w, int nb, int B, float* g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int cols = NOUT * nb;
    if (i >= (HID + 1) * cols) return;
    const int r = i / cols, col = i % cols, k = col / NOUT, c = col % NOUT;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += (w ? w[b * nb + k] : 1.0f) * geff[(int64_t(b) * (HID + 1) + r) * NOUT + c];
    g[int64_t(r) * cols + col] = s;
}

// P1 in the projection's kappa order: [mt][s][g][t][e] = P1[kappa(s, g, e)][32 mt + t]
__global__ void k_p1_kappa(const float* p1, bf16* dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C * HID) return;
    const int e = i & 7, t = (i >> 3) & 31, g = (i >> 8) & 1, s = (i >> 9) & 1, mt = i >> 10;
    dst[i] = (bf16)p1[kappa(s, g, e) * HID + 32 * mt + t];
}

__global__ void k_to_bf16(const float* src, bf16* dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (bf16)src[i];
}

// Adam with bias correction (Kingma and Ba, Algorithm 1).  The factors
// 1 - b1 and 1 - b2 come in rounded from float64: formed in float32 from the
// rounded b2 = 0.999 they would be off by 1.3e-5 relative.
__global__ void k_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float omb1,
                       float b2, float omb2, float eps, float bc1, float bc2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---- device-side training loop (tf_fno_train, tf_fno_eval) ----

// Per-block float64 sums of squares over n floats (fixed grid, so the
// partials and their host sum in block order are deterministic).
constexpr int SQ_BLOCKS = 2048;
__global__ __launch_bounds__(256) void k_sumsq32(const float* x, int64_t n, double* part) {
    double s = 0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(SQ_BLOCKS) * 256) {
        const double v = x[i];
        s += v * v;
    }
    __shared__ double r[256];
    r[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = r[0];
}

// Minibatch gather: sample b of the batch is row idx[b] of the data set;
// targets are multiplied by tscale on the way (grid: (blocks, B)).
__global__ __launch_bounds__(256) void k_gather_targets(const float* y, const int* idx, float tscale, float* yb) {
    const int b = blockIdx.y;
    const float4* src = reinterpret_cast<const float4*>(y + int64_t(idx[b]) * OUT_SZ);
    float4* dst = reinterpret_cast<float4*>(yb + int64_t(b) * OUT_SZ);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < OUT_SZ / 4; i += int64_t(gridDim.x) * 256) {
        float4 v = src[i];
        v.x *= tscale; v.y *= tscale; v.z *= tscale; v.w *= tscale;
        dst[i] = v;
    }
}
__global__ void k_gather_rows(const float* p, const float* w, const int* idx, int B, int nb, float* pb, float* wb) {
    for (int i = threadIdx.x; i < B * NPAR; i += blockDim.x) pb[i] = p[int64_t(idx[i / NPAR]) * NPAR + i % NPAR];
    if (w)
        for (int i = threadIdx.x; i < B * nb; i += blockDim.x) wb[i] = w[int64_t(idx[i / nb]) * nb + i % nb];
}
__global__ void k_log_loss(const double* res, double* log, int step) { log[step] = res[0]; }
__global__ void k_scale(float* x, int64_t n, float s) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= s;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

using host::fail;

inline Ix plain(int s) { return Ix{30, 0, s}; }
inline Ix two(int sh, int hi, int lo) { return Ix{sh, hi, lo}; }

// largest element offset an operand touches (all strides non-negative)
inline int64_t max_ix(Ix a, int n) {
    if (n <= 0) return 0;
    const int64_t mask = (int64_t(1) << a.sh) - 1;
    return int64_t((n - 1) >> a.sh) * a.hi + std::min<int64_t>(n - 1, mask) * a.lo;
}

typedef void (*GemmLaunch)(const GemmArgs&, int, int, hipStream_t);

template <int BM, int BN, int NW, typename TA, typename TB, bool SPLIT>
void launch(const GemmArgs& g, int by, int bz, hipStream_t st) {
    const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((k_gemm<BM, BN, NW, TA, TB, SPLIT>), dim3(tiles, by, bz), dim3(64 * NW), 0, st, g);
}

struct Gemm {
    GemmArgs g;
    int by, bz;
    GemmLaunch fn;
};

// Checks an operand against the size of the buffer it addresses.
inline bool fits(const Operand& o, int rows, int cols, int by, int bz, int64_t size) {
    if (!o.p) return true;
    const int r = std::min(rows, o.ones_from);
    if (r <= 0) return true;
    const int64_t mx = int64_t(by - 1) * o.b1 + int64_t(bz - 1) * o.b2 + max_ix(o.r, r) + max_ix(o.c, cols);
    return mx < size;
}
inline bool fits(const Result& o, int rows, int cols, int by, int bz, int64_t size) {
    const int64_t mx = int64_t(by - 1) * o.b1 + int64_t(bz - 1) * o.b2 + max_ix(o.r, rows) + max_ix(o.c, cols);
    return mx < size;
}

inline Operand opnd(const void* p, Ix r, Ix c, int64_t b1, int64_t b2, int fast_k, int ones_from = 1 << 30) {
    return Operand{p, b1, b2, r, c, ones_from, fast_k, 0};
}

// Whether groups of 4 along the operand's contiguous index are contiguous and
// aligned for 4-element loads (rows x cols is the operand's shape).  Rows
// from ones_from on are never loaded (stage takes them first), so they do
// not bar the vector loads of the others.
inline bool vec_ok(const Operand& o, int rows, int cols, bool is_b, size_t elem) {
    if (!o.p || !o.fast_k) return false;
    const bool k_is_row = is_b;                 // A: (M, K); B: (K, N)
    const Ix fast = o.fast_k ? (k_is_row ? o.r : o.c) : (k_is_row ? o.c : o.r);
    const Ix slow = o.fast_k ? (k_is_row ? o.c : o.r) : (k_is_row ? o.r : o.c);
    const int fext = o.fast_k ? (k_is_row ? rows : cols) : (k_is_row ? cols : rows);
    auto mult4 = [](int64_t v) { return v % 4 == 0; };
    if (fast.lo != 1 || fast.sh < 2 || fext % 4) return false;
    if (fast.sh < 30 && !mult4(fast.hi)) return false;
    if (!mult4(slow.lo) || (slow.sh < 30 && !mult4(slow.hi))) return false;
    if (!mult4(o.b1) || !mult4(o.b2)) return false;
    return (uintptr_t)o.p % (4 * elem) == 0;
}
inline Result res(float* p, Ix r, Ix c, int64_t b1, int64_t b2, float alpha = 1.0f, int acc = 0) {
    return Result{p, b1, b2, r, c, alpha, acc};
}

// DFT tables, float64-built from the exact integer phase (j k mod P), for
// the spectral transform of period P >= N: the window extended by zeros to
// P nodes per axis, the kept modes [0, M) (x) and [0, M) U [P - M, P) (y, z)
// of the period-P DFT, and the inverse's 1/P per axis, cut back to the N
// window nodes.  P = N is the plain transform; the backward passes use the
// transposed tables, so they are the exact adjoints for any P.
struct Tables {
    std::vector<float> fx, fxT, gx, gxT, fs, fsT, gs, gsT;
};

inline Tables build_tables(int P) {
    Tables t;
    auto ang = [P](int a, int b) { return 2.0 * M_PI * double((int64_t(a) * b) % P) / P; };
    auto side = [P](int i) { return i < M ? i : P - 2 * M + i; };
    t.fx.assign(24 * N, 0.f);
    t.gx.assign(N * 24, 0.f);
    for (int kx = 0; kx < M; ++kx)
        for (int x = 0; x < N; ++x) {
            const double th = ang(kx, x), mult = kx == 0 ? 1.0 : 2.0;
            t.fx[(0 * M + kx) * N + x] = float(std::cos(th));
            t.fx[(1 * M + kx) * N + x] = float(-std::sin(th));
            t.gx[x * 24 + 0 * M + kx] = float(mult / P * std::cos(th));
            t.gx[x * 24 + 1 * M + kx] = float(-mult / P * std::sin(th));
        }
    t.fs.assign(48 * 128, 0.f);
    t.gs.assign(128 * 48, 0.f);
    for (int ki = 0; ki < KS; ++ki)
        for (int n = 0; n < N; ++n) {
            const double th = ang(side(ki), n);
            const double fr = std::cos(th), fi = -std::sin(th);       // e^{-i th}
            const double gr = std::cos(th) / P, gi = std::sin(th) / P; // e^{+i th} / P
            // forward block [[fr, -fi], [fi, fr]] at (row (ki, s'), col (n, s))
            t.fs[(2 * ki + 0) * 128 + 2 * n + 0] = float(fr);
            t.fs[(2 * ki + 0) * 128 + 2 * n + 1] = float(-fi);
            t.fs[(2 * ki + 1) * 128 + 2 * n + 0] = float(fi);
            t.fs[(2 * ki + 1) * 128 + 2 * n + 1] = float(fr);
            // inverse block at (row (n, s), col (ki, s'))
            t.gs[(2 * n + 0) * 48 + 2 * ki + 0] = float(gr);
            t.gs[(2 * n + 0) * 48 + 2 * ki + 1] = float(-gi);
            t.gs[(2 * n + 1) * 48 + 2 * ki + 0] = float(gi);
            t.gs[(2 * n + 1) * 48 + 2 * ki + 1] = float(gr);
        }
    auto tr = [](const std::vector<float>& a, int r, int c) {
        std::vector<float> o(a.size());
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < c; ++j) o[j * r + i] = a[i * c + j];
        return o;
    };
    t.fxT = tr(t.fx, 24, N);
    t.gxT = tr(t.gx, N, 24);
    t.fsT = tr(t.fs, 48, 128);
    t.gsT = tr(t.gs, 128, 48);
    return t;
}

}  // namespace fno
}  // namespace tf

using namespace tf::fno;
using tf::host::fail;

struct tf_fno {
    int dev = 0;
    hipStream_t st = nullptr;   // the caller's stream
    hipStream_t cur = nullptr;  // stream launches go to (st, or cap while capturing)
    hipStream_t cap = nullptr;  // private stream inference graphs are captured on
    hipGraphExec_t exec = nullptr;
    const float* g_params = nullptr;
    float* g_out = nullptr;
    int g_batch = 0;
    int maxB = 0;
    int nb = 1;                 // basis fields of the output head
    int64_t np = 0;             // parameter count
    const float* g_w = nullptr;
    bool training = false;
    int64_t adam_t = 0;
    bool working_stale = true;

    std::vector<void*> allocs;
    float *prm = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
    bf16 *wb[LAYERS] = {}, *rb[LAYERS] = {}, *p1b = nullptr, *p2e = nullptr, *p1k = nullptr, *p2k = nullptr;
    float *c2e = nullptr, *geff = nullptr;
    float *fx, *fxT, *gx, *gxT, *fs, *fsT, *gs, *gsT;
    float* tab = nullptr;       // the eight tables, one allocation
    int period = N;             // period of the spectral transform (tables built for it)
    float* V[4] = {};
    float* Z[2] = {};
    float* X3[LAYERS] = {};
    float *T1 = nullptr, *T2 = nullptr, *Y = nullptr, *Y2 = nullptr;
    float *G[2] = {};
    float *out = nullptr, *gout = nullptr, *part = nullptr, *gstar = nullptr;
    bf16 *hT = nullptr, *ghT = nullptr;
    float *pbuf = nullptr, *wbuf = nullptr, *ybuf = nullptr;   // tf_fno_train minibatches (on first use)
    double* dres = nullptr;
    double* lpart = nullptr;

    ~tf_fno() {
        if (st) hipStreamSynchronize(st);
        else hipDeviceSynchronize();
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
        for (void* p : allocs) hipFree(p);
    }

    template <typename T>
    tf_status alloc(T** p, int64_t n) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, size_t(n) * sizeof(T));
        if (e != hipSuccess) return fail(TF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *p = (T*)q;
        return TF_OK;
    }
};

namespace {

constexpr int LOSS_CH = 64;

#define TRY(x)                           \
    do {                                 \
        tf_status s_ = (x);              \
        if (s_ != TF_OK) return s_;      \
    } while (0)

tf_status launched() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return TF_OK;
}

tf_status run(tf_fno* f, Gemm g, int64_t sa, int64_t sb, int64_t sc, size_t ea = 4, size_t eb = 4) {
    if (!fits(g.g.a, g.g.M, g.g.K, g.by, g.bz, sa) || !fits(g.g.b, g.g.K, g.g.N, g.by, g.bz, sb) ||
        !fits(g.g.c, g.g.M, g.g.N, g.by, g.bz, sc))
        return fail(TF_EINVAL, "internal: GEMM operand exceeds its buffer");
    g.g.a.vec = vec_ok(g.g.a, g.g.M, g.g.K, false, ea);
    g.g.b.vec = vec_ok(g.g.b, g.g.K, g.g.N, true, eb);
    g.fn(g.g, g.by, g.bz, f->cur);
    return launched();
}

// ---- the spectral stages (per sample b = blockIdx.z) ----

// x contraction: out[(s,kx)][(zy,c)] = sum_x A[(s,kx)][x] in[(zy,x,c)]
Gemm g_xcontract(const float* A, const float* in, float* out, int B) {
    GemmArgs g{opnd(A, plain(N), plain(1), 0, 0, 1),
               opnd(in, plain(C), two(5, N * C, 1), 0, NODE_SZ, 0),
               res(out, plain(C), two(5, 2 * LINE, 1), 0, X1_SZ), 24, N * N * C, N};
    return Gemm{g, 1, B, launch<32, 128, 4, float, float, true>};
}
// y contraction (per z): X1 layout in, X2 layout out; A is 48 x 128
Gemm g_ycontract(const float* A, const float* in, float* out, int B) {
    GemmArgs g{opnd(A, plain(128), plain(1), 0, 0, 1),
               opnd(in, plain(LINE), plain(1), int64_t(N) * 2 * LINE, X1_SZ, 0),
               res(out, two(1, N * 2 * LINE, LINE), plain(1), 2 * LINE, X2_SZ), 48, LINE, 128};
    return Gemm{g, N, B, launch<64, 128, 4, float, float, true>};
}
// z contraction (per ky): X2 layout in, mode layout out
Gemm g_zcontract(const float* A, const float* in, float* out, int B) {
    GemmArgs g{opnd(A, plain(128), plain(1), 0, 0, 1),
               opnd(in, plain(LINE), plain(1), int64_t(N) * 2 * LINE, X2_SZ, 0),
               res(out, plain(KS * LINE), plain(1), LINE, X3_SZ), 48, LINE, 128};
    return Gemm{g, KS, B, launch<64, 128, 4, float, float, true>};
}
// z expansion (per ky): mode layout in, X2 layout out; A is 128 x 48
Gemm g_zexpand(const float* A, const float* in, float* out, int B) {
    GemmArgs g{opnd(A, plain(48), plain(1), 0, 0, 1),
               opnd(in, plain(KS * LINE), plain(1), LINE, X3_SZ, 0),
               res(out, plain(LINE), plain(1), int64_t(N) * 2 * LINE, X2_SZ), 128, LINE, 48};
    return Gemm{g, KS, B, launch<64, 128, 4, float, float, true>};
}
// y expansion (per z): X2 layout in, X1 layout out
Gemm g_yexpand(const float* A, const float* in, float* out, int B) {
    GemmArgs g{opnd(A, plain(48), plain(1), 0, 0, 1),
               opnd(in, two(1, N * 2 * LINE, LINE), plain(1), 2 * LINE, X2_SZ, 0),
               res(out, plain(LINE), plain(1), int64_t(N) * 2 * LINE, X1_SZ), 128, LINE, 48};
    return Gemm{g, N, B, launch<64, 128, 4, float, float, true>};
}

// ---- per-mode complex channel mixing as real 64 x 64 blocks ----
// mode q = kz * 288 + (ky * 12 + kx): blockIdx.y = ky * 12 + kx, blockIdx.z = kz
constexpr int64_t MODE_Y = C, MODE_Z = 2 * KS * LINE;

// Y*[b][(s',o)] = sum X*[b][(s,c)] Wq[(s,c)][(s',o)]  (trans: Wq^T)
Gemm g_mix(const float* X, const bf16* R, float* Yo, int B, bool trans) {
    const Ix rr = trans ? plain(1) : plain(64), rc = trans ? plain(64) : plain(1);
    GemmArgs g{opnd(X, plain(X3_SZ), two(5, KS * LINE, 1), MODE_Y, MODE_Z, 1),
               opnd(R, rr, rc, 4096, int64_t(KS * M) * 4096, trans ? 1 : 0),
               res(Yo, plain(X3_SZ), two(5, KS * LINE, 1), MODE_Y, MODE_Z), B, 64, 64};
    // the adjoint (trans) splits the gradient operand into bf16 hi + lo; the
    // forward keeps one bf16 copy of the modes
    return Gemm{g, KS * M, KS, trans ? launch<32, 64, 2, float, bf16, true> : launch<32, 64, 2, float, bf16, false>};
}
// G*[q][(s,c)][(s',o)] = sum_b X*[b][(s,c)] gY*[b][(s',o)]
Gemm g_mix_grad(const float* X, const float* gY, float* gs, int B) {
    GemmArgs g{opnd(X, two(5, KS * LINE, 1), plain(X3_SZ), MODE_Y, MODE_Z, 0),
               opnd(gY, plain(X3_SZ), two(5, KS * LINE, 1), MODE_Y, MODE_Z, 0),
               res(gs, plain(64), plain(1), 4096, int64_t(KS * M) * 4096), 64, 64, B};
    return Gemm{g, KS * M, KS, launch<64, 64, 4, float, float, true>};
}

}  // namespace

extern "C" {

int64_t tf_fno_param_count(int32_t nbasis) {
    return (nbasis == 1 || nbasis == 2 || nbasis == 4) ? nparams(nbasis) : -1;
}

tf_status tf_fno_phasor_weights(const tf_pulse* pulse, int32_t nbasis, double* w) {
    if (!w) return fail(TF_EINVAL, "w is NULL");
    if (nbasis != 1 && nbasis != 2 && nbasis != 4) return fail(TF_EINVAL, "nbasis must be 1, 2 or 4");
    TRY(tf::host::validate_pulse(pulse));
    if (nbasis == 1) {
        w[0] = 1.0;
        return TF_OK;
    }
    // envelope Re[exp(i sig phase) G]: sig = +1 spectral, -1 for the sin(k z - phase) envelopes
    const double sig = pulse->envelope == TF_ENV_SPECTRAL ? 1.0 : -1.0;
    double gnorm = 1.0;
    if (pulse->envelope == TF_ENV_SPECTRAL) {
        std::vector<double> tab;
        tf::host::spectral_table(pulse, tab, gnorm);
        if (!(gnorm > 0.0)) return fail(TF_EINVAL, "spectral pulse vanishes in its window");
    }
    const double zr = std::cos(sig * pulse->cep), zi = std::sin(sig * pulse->cep);
    if (nbasis == 2) {
        w[0] = zr / gnorm;
        w[1] = -zi / gnorm;
        return TF_OK;
    }
    double ar = 1.0, ai = 0.0, br = 0.0, bi = 0.0;
    if (pulse->polarization == TF_POL_LINEAR) {
        const double e = pulse->ellipticity, n = std::sqrt(1.0 + e * e);
        const double c = std::cos(pulse->pol_angle), s = std::sin(pulse->pol_angle);
        ar = c / n; ai = -sig * e * s / n;
        br = s / n; bi = sig * e * c / n;
    }
    w[0] = (zr * ar - zi * ai) / gnorm;     // Re(z a)
    w[1] = -(zr * ai + zi * ar) / gnorm;    // -Im(z a)
    w[2] = (zr * br - zi * bi) / gnorm;
    w[3] = -(zr * bi + zi * br) / gnorm;
    return TF_OK;
}

// Builds the DFT tables of period P and copies them into f->tab (synchronous).
static tf_status upload_tables(tf_fno* f, int P) {
    Tables t = build_tables(P);
    std::vector<float> all;
    auto put = [&](const std::vector<float>& v, float** p) {
        *p = f->tab + all.size();
        all.insert(all.end(), v.begin(), v.end());
    };
    put(t.fx, &f->fx); put(t.fxT, &f->fxT); put(t.gx, &f->gx); put(t.gxT, &f->gxT);
    put(t.fs, &f->fs); put(t.fsT, &f->fsT); put(t.gs, &f->gs); put(t.gsT, &f->gsT);
    TF_HIP(hipMemcpyAsync(f->tab, all.data(), all.size() * sizeof(float), hipMemcpyHostToDevice, f->st));
    TF_HIP(hipStreamSynchronize(f->st));
    f->period = P;
    return TF_OK;
}

tf_status tf_fno_set_period(tf_fno* f, int32_t period) {
    if (!f) return fail(TF_EINVAL, "NULL argument");
    if (period < N || period > 4 * N) return fail(TF_EINVAL, "period must be in [64, 256]");
    if (period == f->period) return TF_OK;
    TF_HIP(hipSetDevice(f->dev));
    TF_HIP(hipStreamSynchronize(f->st));
    return upload_tables(f, period);
}

tf_status tf_fno_get_period(const tf_fno* f, int32_t* period) {
    if (!f || !period) return fail(TF_EINVAL, "NULL argument");
    *period = f->period;
    return TF_OK;
}

tf_status tf_fno_create(int32_t max_batch, int32_t training, int32_t nbasis, void* hip_stream, tf_fno** out) {
    if (!out) return fail(TF_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_batch < 1 || max_batch > 128) return fail(TF_EINVAL, "max_batch must be in [1, 128]");
    if (nbasis != 1 && nbasis != 2 && nbasis != 4) return fail(TF_EINVAL, "nbasis must be 1, 2 or 4");
    std::unique_ptr<tf_fno> f(new tf_fno());
    f->nb = nbasis;
    f->np = nparams(nbasis);
    f->maxB = max_batch;
    f->training = training != 0;
    f->st = (hipStream_t)hip_stream;
    f->cur = f->st;
    TF_HIP(hipGetDevice(&f->dev));
    TF_HIP(hipStreamCreateWithFlags(&f->cap, hipStreamNonBlocking));
    const int64_t B = max_batch;

    const int64_t NPARAMS = f->np;
    TRY(f->alloc(&f->prm, NPARAMS));
    TF_HIP(hipMemset(f->prm, 0, NPARAMS * sizeof(float)));
    for (int l = 0; l < LAYERS; ++l) {
        TRY(f->alloc(&f->wb[l], C * C));
        TRY(f->alloc(&f->rb[l], int64_t(NMODES) * 4096));
    }
    TRY(f->alloc(&f->p1b, C * HID));
    TRY(f->alloc(&f->p2e, B * HID * NOUT));
    TRY(f->alloc(&f->c2e, B * NOUT));
    TRY(f->alloc(&f->p1k, C * HID));
    TRY(f->alloc(&f->p2k, B * KSLOTS));
    TF_HIP(hipMemset(f->p2k, 0, B * KSLOTS * sizeof(bf16)));     // rows t >= 6 stay 0

    const int64_t ntab = 4 * 24 * N + 4 * 48 * 128;
    TRY(f->alloc(&f->tab, ntab));
    TRY(upload_tables(f.get(), N));

    TRY(f->alloc(&f->V[0], B * NODE_SZ));
    TRY(f->alloc(&f->V[1], B * NODE_SZ));
    TRY(f->alloc(&f->T1, B * X1_SZ));
    TRY(f->alloc(&f->T2, B * X2_SZ));
    TRY(f->alloc(&f->X3[0], B * X3_SZ));
    TRY(f->alloc(&f->Y, B * X3_SZ));
    TRY(f->alloc(&f->out, B * OUT_SZ));
    TRY(f->alloc(&f->dres, 1 + 2 * B));      // loss, per-sample scales, per-sample ratios
    TRY(f->alloc(&f->lpart, B * LOSS_CH * 2));
    if (f->training) {
        TRY(f->alloc(&f->grad, NPARAMS));
        TRY(f->alloc(&f->am, NPARAMS));
        TRY(f->alloc(&f->av, NPARAMS));
        TF_HIP(hipMemset(f->am, 0, NPARAMS * sizeof(float)));
        TF_HIP(hipMemset(f->av, 0, NPARAMS * sizeof(float)));
        TRY(f->alloc(&f->V[2], B * NODE_SZ));
        TRY(f->alloc(&f->V[3], B * NODE_SZ));
        TRY(f->alloc(&f->Z[0], B * NODE_SZ));
        TRY(f->alloc(&f->Z[1], B * NODE_SZ));
        TRY(f->alloc(&f->G[0], B * NODE_SZ));
        TRY(f->alloc(&f->G[1], B * NODE_SZ));
        TRY(f->alloc(&f->X3[1], B * X3_SZ));
        TRY(f->alloc(&f->X3[2], B * X3_SZ));
        TRY(f->alloc(&f->Y2, B * X3_SZ));
        TRY(f->alloc(&f->gout, B * OUT_SZ));
        TRY(f->alloc(&f->hT, B * HID * N3));
        TRY(f->alloc(&f->ghT, B * HID * N3));
        TRY(f->alloc(&f->part, B * NCHUNK * 33 * HID));
        TRY(f->alloc(&f->gstar, int64_t(NMODES) * 4096));
        TRY(f->alloc(&f->geff, B * (HID + 1) * NOUT));
    }
    TF_HIP(hipDeviceSynchronize());
    *out = f.release();
    return TF_OK;
}

tf_status tf_fno_destroy(tf_fno* f) {
    delete f;
    return TF_OK;
}

}  // extern "C"

namespace {

tf_status refresh_working(tf_fno* f) {
    if (!f->working_stale) return TF_OK;
    for (int l = 0; l < LAYERS; ++l) {
        hipLaunchKernelGGL(k_to_bf16, dim3((C * C + 255) / 256), dim3(256), 0, f->cur, f->prm + off_w(l), f->wb[l],
                           C * C);
        const int64_t n = int64_t(NMODES) * 4096;
        hipLaunchKernelGGL(k_expand_r, dim3((n + 255) / 256), dim3(256), 0, f->cur, f->prm + off_r(l), f->rb[l]);
    }
    hipLaunchKernelGGL(k_to_bf16, dim3((C * HID + 255) / 256), dim3(256), 0, f->cur, f->prm + OFF_P1, f->p1b, C * HID);
    hipLaunchKernelGGL(k_p1_kappa, dim3((C * HID + 255) / 256), dim3(256), 0, f->cur, f->prm + OFF_P1, f->p1k);
    TRY(launched());
    f->working_stale = false;
    return TF_OK;
}

// Forward pass.  Training keeps v_l, z_l and the modes of every layer for the
// backward pass; inference ping-pongs two node tensors.
tf_status forward_infer(tf_fno* f, const float* params, int B, float* out);

tf_status forward_body(tf_fno* f, const float* params, const float* hw, int B, float* out) {
    const int64_t nb = B;
    {
        const int n = B * (HID + 1) * NOUT;
        hipLaunchKernelGGL(k_head_eff, dim3((n + 255) / 256), dim3(256), 0, f->cur, f->prm + OFF_P2,
                           f->prm + off_c2(f->nb), hw, f->nb, B, f->p2e, f->c2e, f->p2k);
    }
    if (!f->training) return forward_infer(f, params, B, out);
    {
        const int64_t tot = nb * NODE_SZ;
        hipLaunchKernelGGL(k_lift, dim3((tot + 255) / 256), dim3(256), 0, f->cur, params, f->prm + OFF_W0,
                           f->prm + OFF_B0, f->V[0], tot);
        TRY(launched());
    }
    const int64_t szN = nb * NODE_SZ, sz1 = nb * X1_SZ, sz2 = nb * X2_SZ, sz3 = nb * X3_SZ;
    float* v = f->V[0];
    for (int l = 0; l < LAYERS; ++l) {
        float* modes = f->training ? f->X3[l] : f->X3[0];
        TRY(run(f, g_xcontract(f->fx, v, f->T1, B), 24 * N, szN, sz1));
        TRY(run(f, g_ycontract(f->fs, f->T1, f->T2, B), 48 * 128, sz1, sz2));
        TRY(run(f, g_zcontract(f->fs, f->T2, modes, B), 48 * 128, sz2, sz3));
        TRY(run(f, g_mix(modes, f->rb[l], f->Y, B, false), sz3, int64_t(NMODES) * 4096, sz3, 4, 2));
        TRY(run(f, g_zexpand(f->gs, f->Y, f->T2, B), 128 * 48, sz3, sz2));
        TRY(run(f, g_yexpand(f->gs, f->T2, f->T1, B), 128 * 48, sz2, sz1));
        float* nv = f->training ? f->V[l + 1] : (v == f->V[0] ? f->V[1] : f->V[0]);
        LineArgs a{f->gx, f->T1, v, f->wb[l], f->prm + off_b(l), nullptr,
                   (f->training && l < LAYERS - 1) ? f->Z[l] : nullptr, nv, B * N * N, 0, l < LAYERS - 1};
        hipLaunchKernelGGL(k_lineout, dim3((B * N * N + 3) / 4), dim3(256), 0, f->cur, a);
        TRY(launched());
        v = nv;
    }
    ProjArgs p{v, f->p1b, f->prm + OFF_C1, f->p2e, f->c2e, out, nullptr, nullptr, nullptr, nullptr,
               B * (N3 / 32), 0};
    hipLaunchKernelGGL(k_proj, dim3((p.ntiles + 3) / 4), dim3(256), 0, f->cur, p);
    return launched();
}

// Inference: lift + first x contraction, then per layer the y and z
// contractions, mixing and expansions, and one fused x-line kernel.
tf_status forward_infer(tf_fno* f, const float* params, int B, float* out) {
    const int64_t nb = B;
    const int64_t sz1 = nb * X1_SZ, sz2 = nb * X2_SZ, sz3 = nb * X3_SZ;
    const int lines = B * N * N;
    InfArgs a{f->gx, f->fx, f->T1, nullptr, params, f->prm + OFF_W0, f->prm + OFF_B0, nullptr, nullptr,
              nullptr, f->T1, f->p1k, f->prm + OFF_C1, f->p2k, f->c2e, out, lines};
    hipLaunchKernelGGL(k_lift_x, dim3((lines + 3) / 4), dim3(256), 0, f->cur, a);
    TRY(launched());
    const float* v = nullptr;                 // v_0 is recomputed, never stored
    for (int l = 0; l < LAYERS; ++l) {
        TRY(run(f, g_ycontract(f->fs, f->T1, f->T2, B), 48 * 128, sz1, sz2));
        TRY(run(f, g_zcontract(f->fs, f->T2, f->X3[0], B), 48 * 128, sz2, sz3));
        TRY(run(f, g_mix(f->X3[0], f->rb[l], f->Y, B, false), sz3, int64_t(NMODES) * 4096, sz3, 4, 2));
        TRY(run(f, g_zexpand(f->gs, f->Y, f->T2, B), 128 * 48, sz3, sz2));
        TRY(run(f, g_yexpand(f->gs, f->T2, f->T1, B), 128 * 48, sz2, sz1));
        a.act = v;
        a.w = f->wb[l];
        a.bias = f->prm + off_b(l);
        if (l < LAYERS - 1) {
            float* nv = (v == f->V[0]) ? f->V[1] : f->V[0];
            a.vout = nv;
            hipLaunchKernelGGL(k_line_fwd, dim3((lines + 3) / 4), dim3(256), 0, f->cur, a);
            v = nv;
        } else {
            hipLaunchKernelGGL(k_line_proj, dim3((2 * lines + 3) / 4), dim3(256), 0, f->cur, a);
        }
        TRY(launched());
    }
    return TF_OK;
}

tf_status forward(tf_fno* f, const float* params, const float* hw, int B, float* out) {
    TRY(refresh_working(f));
    return forward_body(f, params, hw, B, out);
}

// split-K weight gradient [A | 1]^T-style reductions into the flat gradient
tf_status reduce_into(tf_fno* f, int nparts, int len, float* dst, int groups = 1) {
    hipLaunchKernelGGL(k_reduce, dim3((len + 63) / 64, groups), dim3(256), 0, f->cur, f->part, nparts, len, dst);
    return launched();
}

// Backward pass.  The weight-gradient GEMMs and the adjoint of the mixing
// take their float32 operands as bf16 hi + lo parts (three MFMAs, about
// float32 products): a one-part bf16 copy of each activation would put a
// relative error of up to 2^-9 on every term of sums that cancel heavily.
// The bf16 weights themselves are exact in either form.
tf_status backward(tf_fno* f, const float* params, const float* hw, const float* target, int B) {
    const int64_t nb = B;
    const int64_t szN = nb * NODE_SZ, sz1 = nb * X1_SZ, sz2 = nb * X2_SZ, sz3 = nb * X3_SZ;
    const int64_t szO = nb * OUT_SZ, szH = nb * HID * N3, szP = nb * NCHUNK * 33 * HID;
    // loss and dL/dout
    hipLaunchKernelGGL(k_loss_part, dim3(LOSS_CH, B), dim3(256), 0, f->cur, f->out, target, f->lpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(LOSS_THREADS), 0, f->cur, f->lpart, LOSS_CH, B, f->dres,
                       f->dres + 1 + B);
    hipLaunchKernelGGL(k_gout, dim3((szO + 255) / 256), dim3(256), 0, f->cur, f->out, target, f->dres, f->gout, szO);
    TRY(launched());
    // projection
    float* g = f->G[0];
    ProjArgs p{f->V[3], f->p1b, f->prm + OFF_C1, f->p2e, f->c2e, nullptr, f->gout, g, f->hT, f->ghT,
               B * (N3 / 32), 1};
    hipLaunchKernelGGL(k_proj, dim3((p.ntiles + 3) / 4), dim3(256), 0, f->cur, p);
    TRY(launched());
    {   // [P1; c1] = [v3 | 1]^T dL/dpre
        GemmArgs a{opnd(f->V[3], plain(1), plain(C), int64_t(CHUNK) * C, NODE_SZ, 0, C),
                   opnd(f->ghT, plain(1), plain(N3), CHUNK, int64_t(HID) * N3, 1),
                   res(f->part, plain(HID), plain(1), 33 * HID, int64_t(NCHUNK) * 33 * HID), 33, HID, CHUNK};
        TRY(run(f, Gemm{a, NCHUNK, B, launch<64, 128, 4, float, bf16, true>}, szN, szH, szP, 4, 2));
        TRY(reduce_into(f, B * NCHUNK, 33 * HID, f->grad + OFF_P1));
    }
    {   // [P2; c2] = [h | 1]^T dL/dout
        GemmArgs a{opnd(f->hT, plain(N3), plain(1), CHUNK, int64_t(HID) * N3, 1, HID),
                   opnd(f->gout, plain(1), plain(N3), CHUNK, OUT_SZ, 1),
                   res(f->part, plain(NOUT), plain(1), 129 * NOUT, int64_t(NCHUNK) * 129 * NOUT), 129, NOUT, CHUNK};
        TRY(run(f, Gemm{a, NCHUNK, B, launch<32, 32, 1, bf16, float, true>}, szH, szO, szP, 2, 4));
        // per-sample gradient of the effective head, then through the head weights
        TRY(reduce_into(f, NCHUNK, 129 * NOUT, f->geff, B));
        const int n = (HID + 1) * NOUT * f->nb;
        hipLaunchKernelGGL(k_head_grad, dim3((n + 255) / 256), dim3(256), 0, f->cur, f->geff, hw, f->nb, B,
                           f->grad + OFF_P2);
        TRY(launched());
    }
    for (int l = LAYERS - 1; l >= 0; --l) {
        float* gn = g == f->G[0] ? f->G[1] : f->G[0];
        {   // [W_l; b_l] = [v_l | 1]^T dL/dz_l
            GemmArgs a{opnd(f->V[l], plain(1), plain(C), int64_t(CHUNK) * C, NODE_SZ, 0, C),
                       opnd(g, plain(C), plain(1), int64_t(CHUNK) * C, NODE_SZ, 0),
                       res(f->part, plain(C), plain(1), 33 * C, int64_t(NCHUNK) * 33 * C), 33, C, CHUNK};
            TRY(run(f, Gemm{a, NCHUNK, B, launch<64, 32, 2, float, float, true>}, szN, szN, szP));
            TRY(reduce_into(f, B * NCHUNK, 33 * C, f->grad + off_w(l)));
        }
        // adjoint of the inverse transform: modes gradient
        TRY(run(f, g_xcontract(f->gxT, g, f->T1, B), 24 * N, szN, sz1));
        TRY(run(f, g_ycontract(f->gsT, f->T1, f->T2, B), 48 * 128, sz1, sz2));
        TRY(run(f, g_zcontract(f->gsT, f->T2, f->Y, B), 48 * 128, sz2, sz3));
        // mixing: dR and dX
        TRY(run(f, g_mix_grad(f->X3[l], f->Y, f->gstar, B), sz3, sz3, int64_t(NMODES) * 4096));
        {
            const int64_t n = int64_t(NMODES) * C * C;
            hipLaunchKernelGGL(k_fold_r, dim3((n + 255) / 256), dim3(256), 0, f->cur, f->gstar, f->grad + off_r(l));
            TRY(launched());
        }
        TRY(run(f, g_mix(f->Y, f->rb[l], f->Y2, B, true), sz3, int64_t(NMODES) * 4096, sz3, 4, 2));
        // adjoint of the forward transform, then the x line with the pointwise branch
        TRY(run(f, g_zexpand(f->fsT, f->Y2, f->T2, B), 128 * 48, sz3, sz2));
        TRY(run(f, g_yexpand(f->fsT, f->T2, f->T1, B), 128 * 48, sz2, sz1));
        LineArgs a{f->fxT, f->T1, g, f->wb[l], nullptr, l > 0 ? f->Z[l - 1] : nullptr, nullptr, gn, B * N * N, 1, 0};
        hipLaunchKernelGGL(k_lineout, dim3((B * N * N + 3) / 4), dim3(256), 0, f->cur, a);
        TRY(launched());
        g = gn;
    }
    hipLaunchKernelGGL(k_lift_grad_part, dim3(N, B), dim3(256), 0, f->cur, g, f->part);
    hipLaunchKernelGGL(k_lift_grad_final, dim3(1), dim3(LIFT_THREADS), 0, f->cur, f->part, params, B, f->grad);
    return launched();
}

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014): the shuffles' generator.
uint64_t splitmix64(uint64_t& st) {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Device buffers of one call, freed on every return path after the stream
// has drained.
struct CallBuffers {
    hipStream_t st;
    std::vector<void*> ptrs;
    explicit CallBuffers(hipStream_t s) : st(s) {}
    ~CallBuffers() {
        if (!ptrs.empty()) (void)hipStreamSynchronize(st);
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    tf_status alloc(T** p, int64_t n) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, size_t(n) * sizeof(T));
        if (e != hipSuccess) return fail(TF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        ptrs.push_back(q);
        *p = static_cast<T*>(q);
        return TF_OK;
    }
};

tf_status check_batch(tf_fno* f, int B, const float* hw, bool need_w = true) {
    if (!f) return fail(TF_EINVAL, "surrogate is NULL");
    if (B < 1 || B > f->maxB) return fail(TF_EINVAL, "batch must be in [1, max_batch]");
    if (need_w && !hw && f->nb != 1) return fail(TF_EINVAL, "a head of several basis fields needs its weights");
    TF_HIP(hipSetDevice(f->dev));
    return TF_OK;
}

}  // namespace

extern "C" {

tf_status tf_fno_set_params(tf_fno* f, const float* src, int32_t src_on_device) {
    if (!f || !src) return fail(TF_EINVAL, "NULL argument");
    const int64_t NPARAMS = f->np;
    TF_HIP(hipSetDevice(f->dev));
    TF_HIP(hipMemcpyAsync(f->prm, src, NPARAMS * sizeof(float),
                          src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, f->st));
    if (f->training) {
        TF_HIP(hipMemsetAsync(f->am, 0, NPARAMS * sizeof(float), f->st));
        TF_HIP(hipMemsetAsync(f->av, 0, NPARAMS * sizeof(float), f->st));
    }
    f->adam_t = 0;
    f->working_stale = true;
    if (!src_on_device) TF_HIP(hipStreamSynchronize(f->st));
    return TF_OK;
}

tf_status tf_fno_get_params(tf_fno* f, float* dst, int32_t dst_on_device) {
    if (!f || !dst) return fail(TF_EINVAL, "NULL argument");
    const int64_t NPARAMS = f->np;
    TF_HIP(hipSetDevice(f->dev));
    TF_HIP(hipMemcpyAsync(dst, f->prm, NPARAMS * sizeof(float),
                          dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, f->st));
    if (!dst_on_device) TF_HIP(hipStreamSynchronize(f->st));
    return TF_OK;
}

tf_status tf_fno_forward(tf_fno* f, const float* params, const float* head_w, int32_t batch, float* out) {
    TRY(check_batch(f, batch, head_w));
    if (!params || !out) return fail(TF_EINVAL, "NULL argument");
    return forward(f, params, head_w, batch, out);
}

tf_status tf_fno_infer(tf_fno* f, const float* params, const float* head_w, int32_t batch, float* out) {
    TRY(check_batch(f, batch, head_w));
    if (!params || !out) return fail(TF_EINVAL, "NULL argument");
    TRY(refresh_working(f));
    if (!f->exec || f->g_params != params || f->g_w != head_w || f->g_out != out || f->g_batch != batch) {
        if (f->exec) {
            TF_HIP(hipStreamSynchronize(f->st));
            TF_HIP(hipGraphExecDestroy(f->exec));
            f->exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        TF_HIP(hipStreamBeginCapture(f->cap, hipStreamCaptureModeThreadLocal));
        f->cur = f->cap;
        const tf_status st = forward_body(f, params, head_w, batch, out);
        f->cur = f->st;
        const hipError_t e = hipStreamEndCapture(f->cap, &graph);
        if (st != TF_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return st != TF_OK ? st : fail(TF_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        }
        const hipError_t e2 = hipGraphInstantiate(&f->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) {
            f->exec = nullptr;
            return fail(TF_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e2));
        }
        f->g_params = params;
        f->g_w = head_w;
        f->g_out = out;
        f->g_batch = batch;
    }
    TF_HIP(hipGraphLaunch(f->exec, f->st));
    return TF_OK;
}

tf_status tf_fno_loss_grad(tf_fno* f, const float* params, const float* head_w, const float* target, int32_t batch,
                           double* loss, float* grad) {
    TRY(check_batch(f, batch, head_w));
    if (!f->training) return fail(TF_ESTATE, "surrogate was created for inference only");
    if (!params || !target) return fail(TF_EINVAL, "NULL argument");
    const int64_t NPARAMS = f->np;
    TRY(forward(f, params, head_w, batch, f->out));
    TRY(backward(f, params, head_w, target, batch));
    if (grad) TF_HIP(hipMemcpyAsync(grad, f->grad, NPARAMS * sizeof(float), hipMemcpyDeviceToHost, f->st));
    if (loss) TF_HIP(hipMemcpyAsync(loss, f->dres, sizeof(double), hipMemcpyDeviceToHost, f->st));
    if (grad || loss) TF_HIP(hipStreamSynchronize(f->st));
    return TF_OK;
}

tf_status tf_fno_train_step(tf_fno* f, const float* params, const float* head_w, const float* target,
                            int32_t batch, double lr, double* loss) {
    if (!(lr >= 0.0) || !std::isfinite(lr)) return fail(TF_EINVAL, "lr must be finite and >= 0");
    TRY(tf_fno_loss_grad(f, params, head_w, target, batch, nullptr, nullptr));
    const int64_t NPARAMS = f->np;
    f->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = float(1.0 - std::pow(b1, double(f->adam_t))), bc2 = float(1.0 - std::pow(b2, double(f->adam_t)));
    hipLaunchKernelGGL(k_adam, dim3((NPARAMS + 255) / 256), dim3(256), 0, f->cur, f->prm, f->am, f->av, f->grad,
                       NPARAMS, float(lr), float(b1), float(1.0 - b1), float(b2), float(1.0 - b2), 1e-8f, bc1, bc2);
    TRY(launched());
    f->working_stale = true;
    if (loss) {
        TF_HIP(hipMemcpyAsync(loss, f->dres, sizeof(double), hipMemcpyDeviceToHost, f->st));
        TF_HIP(hipStreamSynchronize(f->st));
    }
    return TF_OK;
}

tf_status tf_fno_train(tf_fno* f, const float* params, const float* head_w, const float* targets, int64_t n,
                       const tf_train_cfg* cfg, double* final_loss) {
    if (!f || !cfg) return fail(TF_EINVAL, "surrogate and cfg must not be NULL");
    if (!f->training) return fail(TF_ESTATE, "surrogate was created for inference only");
    if (!params || !targets) return fail(TF_EINVAL, "params and targets must not be NULL");
    if (f->nb != 1 && !head_w) return fail(TF_EINVAL, "a head of several basis fields needs its weights");
    const int B = cfg->batch;
    if (B < 1 || B > f->maxB) return fail(TF_EINVAL, "batch must be in [1, max_batch]");
    if (n < B || n > (int64_t(1) << 30)) return fail(TF_EINVAL, "need batch <= n < 2^30");
    if (cfg->epochs < 1) return fail(TF_EINVAL, "epochs must be >= 1");
    if (!std::isfinite(cfg->lr) || cfg->lr < 0.0) return fail(TF_EINVAL, "lr must be finite and >= 0");
    if (!(cfg->lr_min_frac >= 0.0 && cfg->lr_min_frac <= 1.0)) return fail(TF_EINVAL, "lr_min_frac must be in [0, 1]");
    TF_HIP(hipSetDevice(f->dev));
    const int64_t NPARAMS = f->np;
    if (!f->ybuf) {
        TRY(f->alloc(&f->pbuf, int64_t(f->maxB) * NPAR));
        TRY(f->alloc(&f->wbuf, int64_t(f->maxB) * f->nb));
        TRY(f->alloc(&f->ybuf, int64_t(f->maxB) * OUT_SZ));
    }
    const int64_t spe = n / B, total = spe * cfg->epochs;
    CallBuffers cb(f->st);
    int* idx = nullptr;
    double *log = nullptr, *part = nullptr;
    TRY(cb.alloc(&idx, n));
    TRY(cb.alloc(&log, spe));
    TRY(cb.alloc(&part, SQ_BLOCKS));
    // target scale: the root mean square of every target value
    double scale = 1.0;
    if (cfg->scale_targets) {
        hipLaunchKernelGGL(k_sumsq32, dim3(SQ_BLOCKS), dim3(256), 0, f->st, targets, n * OUT_SZ, part);
        TRY(launched());
        std::vector<double> h(SQ_BLOCKS);
        TF_HIP(hipMemcpyAsync(h.data(), part, SQ_BLOCKS * sizeof(double), hipMemcpyDeviceToHost, f->st));
        TF_HIP(hipStreamSynchronize(f->st));
        double ss = 0;
        for (double v : h) ss += v;
        scale = std::sqrt(ss / (double(n) * double(OUT_SZ)));
        if (!(scale > 0.0) || !std::isfinite(scale)) return fail(TF_ENONFINITE, "targets have no finite nonzero RMS");
    }
    const float tscale = float(1.0 / scale);
    std::vector<int> perm(n);
    std::vector<double> hlog(spe);
    uint64_t rng = cfg->seed;
    double last = 0.0;
    f->cur = f->st;
    const double b1 = 0.9, b2 = 0.999;
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        // Fisher-Yates shuffle of the sample order
        for (int64_t i = 0; i < n; ++i) perm[i] = int(i);
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[splitmix64(rng) % uint64_t(i + 1)]);
        TF_HIP(hipMemcpyAsync(idx, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, f->st));
        for (int64_t k = 0; k < spe; ++k) {
            const int* bi = idx + k * B;
            hipLaunchKernelGGL(k_gather_rows, dim3(1), dim3(256), 0, f->st, params, f->nb != 1 ? head_w : nullptr, bi,
                               B, f->nb, f->pbuf, f->wbuf);
            hipLaunchKernelGGL(k_gather_targets, dim3(512, B), dim3(256), 0, f->st, targets, bi, tscale, f->ybuf);
            TRY(launched());
            const float* hw = f->nb != 1 ? f->wbuf : nullptr;
            TRY(forward(f, f->pbuf, hw, B, f->out));
            TRY(backward(f, f->pbuf, hw, f->ybuf, B));
            // cosine decay from lr to lr * lr_min_frac over all steps
            const double step = double(ep) * double(spe) + double(k);
            const double a = cfg->lr * (cfg->lr_min_frac +
                                        (1.0 - cfg->lr_min_frac) * 0.5 * (1.0 + std::cos(M_PI * step / double(total))));
            f->adam_t += 1;
            const float bc1 = float(1.0 - std::pow(b1, double(f->adam_t)));
            const float bc2 = float(1.0 - std::pow(b2, double(f->adam_t)));
            hipLaunchKernelGGL(k_adam, dim3((NPARAMS + 255) / 256), dim3(256), 0, f->st, f->prm, f->am, f->av, f->grad,
                               NPARAMS, float(a), float(b1), float(1.0 - b1), float(b2), float(1.0 - b2), 1e-8f, bc1,
                               bc2);
            hipLaunchKernelGGL(k_log_loss, dim3(1), dim3(1), 0, f->st, f->dres, log, int(k));
            TRY(launched());
            f->working_stale = true;
        }
        TF_HIP(hipMemcpyAsync(hlog.data(), log, spe * sizeof(double), hipMemcpyDeviceToHost, f->st));
        TF_HIP(hipStreamSynchronize(f->st));
        double m = 0;
        for (double v : hlog) m += v;
        last = m / double(spe);
        if (cfg->epoch_loss) cfg->epoch_loss[ep] = last;
        if (cfg->progress) cfg->progress(int32_t(ep), last, cfg->progress_user);
        if (!std::isfinite(last)) return fail(TF_ENONFINITE, "training loss is not finite");
    }
    if (cfg->scale_targets) {
        // fold the scale into the projection so the operator predicts the
        // targets themselves; the Adam moments no longer match: reset them
        const int64_t m = NPARAMS - OFF_P2;
        hipLaunchKernelGGL(k_scale, dim3((m + 255) / 256), dim3(256), 0, f->st, f->prm + OFF_P2, m, float(scale));
        TRY(launched());
        TF_HIP(hipMemsetAsync(f->am, 0, NPARAMS * sizeof(float), f->st));
        TF_HIP(hipMemsetAsync(f->av, 0, NPARAMS * sizeof(float), f->st));
        f->adam_t = 0;
        f->working_stale = true;
    }
    TF_HIP(hipStreamSynchronize(f->st));
    if (final_loss) *final_loss = last;
    return TF_OK;
}

tf_status tf_fno_eval(tf_fno* f, const float* params, const float* head_w, const float* targets, int64_t n,
                      double* rel_l2) {
    if (!f || !params || !targets || !rel_l2) return fail(TF_EINVAL, "NULL argument");
    if (f->nb != 1 && !head_w) return fail(TF_EINVAL, "a head of several basis fields needs its weights");
    if (n < 1 || n > (int64_t(1) << 30)) return fail(TF_EINVAL, "need 1 <= n < 2^30");
    TF_HIP(hipSetDevice(f->dev));
    CallBuffers cb(f->st);
    double* res = nullptr;
    TRY(cb.alloc(&res, n));
    f->cur = f->st;
    for (int64_t i0 = 0; i0 < n; i0 += f->maxB) {
        const int nb = int(std::min<int64_t>(f->maxB, n - i0));
        TRY(forward(f, params + i0 * NPAR, f->nb != 1 ? head_w + i0 * f->nb : nullptr, nb, f->out));
        hipLaunchKernelGGL(k_loss_part, dim3(LOSS_CH, nb), dim3(256), 0, f->st, f->out, targets + i0 * OUT_SZ,
                           f->lpart);
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(LOSS_THREADS), 0, f->st, f->lpart, LOSS_CH, nb, f->dres,
                           f->dres + 1 + nb);
        TRY(launched());
        TF_HIP(hipMemcpyAsync(res + i0, f->dres + 1 + nb, nb * sizeof(double), hipMemcpyDeviceToDevice, f->st));
    }
    TF_HIP(hipMemcpyAsync(rel_l2, res, n * sizeof(double), hipMemcpyDeviceToHost, f->st));
    TF_HIP(hipStreamSynchronize(f->st));
    return TF_OK;
}

tf_status tf_fno_spectral_forward(tf_fno* f, const float* v, int32_t batch, float* modes) {
    TRY(check_batch(f, batch, nullptr, false));
    if (!v || !modes) return fail(TF_EINVAL, "NULL argument");
    const int64_t nb = batch;
    TRY(run(f, g_xcontract(f->fx, v, f->T1, batch), 24 * N, nb * NODE_SZ, nb * X1_SZ));
    TRY(run(f, g_ycontract(f->fs, f->T1, f->T2, batch), 48 * 128, nb * X1_SZ, nb * X2_SZ));
    return run(f, g_zcontract(f->fs, f->T2, modes, batch), 48 * 128, nb * X2_SZ, nb * X3_SZ);
}

tf_status tf_fno_spectral_inverse(tf_fno* f, const float* modes, int32_t batch, float* u) {
    TRY(check_batch(f, batch, nullptr, false));
    if (!modes || !u) return fail(TF_EINVAL, "NULL argument");
    const int64_t nb = batch;
    TRY(run(f, g_zexpand(f->gs, modes, f->T2, batch), 128 * 48, nb * X3_SZ, nb * X2_SZ));
    TRY(run(f, g_yexpand(f->gs, f->T2, f->T1, batch), 128 * 48, nb * X2_SZ, nb * X1_SZ));
    LineArgs a{f->gx, f->T1, nullptr, f->wb[0], nullptr, nullptr, nullptr, u, batch * N * N, 0, 0};
    hipLaunchKernelGGL(k_lineout, dim3((batch * N * N + 3) / 4), dim3(256), 0, f->cur, a);
    return launched();
}

// Checkpoint: magic, version, parameter count, Adam step, then the fp32
// parameters and (when training) the two Adam moments.
tf_status tf_fno_save(tf_fno* f, const char* path) {
    if (!f || !path) return fail(TF_EINVAL, "NULL argument");
    const int64_t NPARAMS = f->np;
    TF_HIP(hipSetDevice(f->dev));
    std::vector<float> h(NPARAMS);
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail(TF_EINVAL, std::string("cannot open ") + path);
    // version 1: the plain transform; version 2 adds the period of the
    // spectral transform as a fifth header word
    const int64_t hdr[5] = {0x4f4e4646554354LL, f->period == N ? 1 : 2, NPARAMS, f->training ? f->adam_t : -1,
                            f->period};
    bool ok = std::fwrite(hdr, sizeof(int64_t), f->period == N ? 4 : 5, fp) == size_t(f->period == N ? 4 : 5);
    const float* srcs[3] = {f->prm, f->am, f->av};
    for (int k = 0; ok && k < (f->training ? 3 : 1); ++k) {
        if (hipMemcpyAsync(h.data(), srcs[k], NPARAMS * sizeof(float), hipMemcpyDeviceToHost, f->st) != hipSuccess ||
            hipStreamSynchronize(f->st) != hipSuccess) {
            std::fclose(fp);
            return fail(TF_EDEVICE, "copy of the parameters failed");
        }
        ok = std::fwrite(h.data(), sizeof(float), NPARAMS, fp) == size_t(NPARAMS);
    }
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? TF_OK : fail(TF_EINVAL, std::string("write failed: ") + path);
}

tf_status tf_fno_load(tf_fno* f, const char* path) {
    if (!f || !path) return fail(TF_EINVAL, "NULL argument");
    const int64_t NPARAMS = f->np;
    TF_HIP(hipSetDevice(f->dev));
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(TF_EINVAL, std::string("cannot open ") + path);
    int64_t hdr[4];
    if (std::fread(hdr, sizeof(hdr), 1, fp) != 1 || hdr[0] != 0x4f4e4646554354LL || (hdr[1] != 1 && hdr[1] != 2) ||
        hdr[2] != NPARAMS) {
        std::fclose(fp);
        return fail(TF_EINVAL, "not a surrogate checkpoint of this architecture");
    }
    int64_t period = N;
    if (hdr[1] == 2 && (std::fread(&period, sizeof(period), 1, fp) != 1 || period < N || period > 4 * N)) {
        std::fclose(fp);
        return fail(TF_EINVAL, "bad period in the surrogate checkpoint");
    }
    std::vector<float> h(NPARAMS);
    float* dsts[3] = {f->prm, f->am, f->av};
    const int nk = (hdr[3] >= 0 && f->training) ? 3 : 1;
    for (int k = 0; k < nk; ++k) {
        if (std::fread(h.data(), sizeof(float), NPARAMS, fp) != size_t(NPARAMS)) {
            std::fclose(fp);
            return fail(TF_EINVAL, "truncated checkpoint");
        }
        hipError_t e = hipMemcpyAsync(dsts[k], h.data(), NPARAMS * sizeof(float), hipMemcpyHostToDevice, f->st);
        if (e == hipSuccess) e = hipStreamSynchronize(f->st);
        if (e != hipSuccess) {
            std::fclose(fp);
            return fail(TF_EDEVICE, std::string("checkpoint upload: ") + hipGetErrorString(e));
        }
    }
    std::fclose(fp);
    if (period != f->period) {
        tf_status st = upload_tables(f, int(period));
        if (st != TF_OK) return st;
    }
    if (f->training) {
        if (nk == 1) {
            TF_HIP(hipMemsetAsync(f->am, 0, NPARAMS * sizeof(float), f->st));
            TF_HIP(hipMemsetAsync(f->av, 0, NPARAMS * sizeof(float), f->st));
        }
        f->adam_t = nk == 3 ? hdr[3] : 0;
    }
    f->working_stale = true;
    TF_HIP(hipStreamSynchronize(f->st));
    return TF_OK;
}

}  // extern "C"
