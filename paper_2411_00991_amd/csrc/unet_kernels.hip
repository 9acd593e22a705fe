// unet_kernels.hip -- BF16 matrix-core kernels of the small U-Net that supplies
// the learned warm start and the block independence proposal.
//
// Every convolution is one implicit GEMM, C[m][n] = sum_k A[m][k] B[n][k], on
// the gfx950 16x16x32 BF16 MFMA with FP32 accumulation.  A workgroup of four
// waves owns a BM x BN tile (waves 2 x 2), stages 32-wide K slices of A and B
// in LDS (double-buffered, rows K-contiguous), and the operand policies below
// generate the addresses of the convolution being computed:
//   forward 3x3:  m = output pixel, k = (tap, c_in),   n = c_out
//   dgrad 3x3:    m = input pixel,  k = (tap', c_out), n = c_in   (flipped taps)
//   wgrad 3x3:    m = c_out,        k = pixel,         n = (tap, c_in)
//   forward 2x2 stride-2 transposed: m = input pixel, k = c_in, n = (i, j, c_out)
//   its dgrad:    m = input pixel,  k = (i, j, c_out),  n = c_in
//   its wgrad:    m = c_in,         k = input pixel,    n = c_out   (per (i, j))
// Activations are NHWC BF16 with a pixel stride `ld` and a channel offset, so
// the skip concatenation is two slices of one buffer.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "unet.h"

namespace bdc {
namespace unet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;          // K slice per step
constexpr int BKP = BK + 8;     // LDS row pitch (bf16): 80 bytes, 16-byte aligned rows
constexpr int NT = 256;         // threads per GEMM workgroup
constexpr int64_t PART_MAX = 1 << 24;   // floats in the caller's split-K partial buffer

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ inline uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ inline void pixel_of(int64_t m, int H, int W, int& b, int& y, int& x) {
    const int64_t hw = (int64_t)H * W;
    b = (int)(m / hw);
    const int r = (int)(m - (int64_t)b * hw);
    y = r / W;
    x = r - y * W;
}

// ---------------------------------------------------------------------------
// Row-major operand policies: prep(row) once per thread, then load(rc, k) gives
// the 8 K-consecutive values of that row at k..k+7 (zero outside).
// ---------------------------------------------------------------------------
struct RowCtx { int64_t pix; int y, x; bool ok; };

// 3x3 neighbourhood gather, k = tap * C + c (C % 8 == 0).
struct OpConv3 {
    Tens t; int64_t M; int K;
    __device__ RowCtx prep(int64_t m) const {
        RowCtx rc; rc.ok = m < M; rc.pix = m; rc.y = rc.x = 0;
        if (rc.ok) { int b; pixel_of(m, t.H, t.W, b, rc.y, rc.x); }
        return rc;
    }
    __device__ uint4 load(const RowCtx& rc, int k) const {
        if (!rc.ok || k >= K) return make_uint4(0, 0, 0, 0);
        const int tap = k / t.C, c = k - tap * t.C;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const int yy = rc.y + dy, xx = rc.x + dx;
        if (yy < 0 || yy >= t.H || xx < 0 || xx >= t.W) return make_uint4(0, 0, 0, 0);
        const int64_t q = rc.pix + (int64_t)dy * t.W + dx;
        return *(const uint4*)(t.p + q * t.ld + t.off + c);
    }
};

// 3x3 gather of a single-channel input, k = tap (< 9), K padded to 16.
struct OpConv3C1 {
    Tens t; int64_t M;
    __device__ RowCtx prep(int64_t m) const { return OpConv3{t, M, 16}.prep(m); }
    __device__ uint4 load(const RowCtx& rc, int k) const {
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int tap = k + e;
            v[e] = 0;
            if (rc.ok && tap < 9) {
                const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                const int yy = rc.y + dy, xx = rc.x + dx;
                if (yy >= 0 && yy < t.H && xx >= 0 && xx < t.W)
                    v[e] = t.p[(rc.pix + (int64_t)dy * t.W + dx) * t.ld + t.off];
            }
        }
        return make_uint4(v[0] | (uint32_t)v[1] << 16, v[2] | (uint32_t)v[3] << 16, v[4] | (uint32_t)v[5] << 16,
                          v[6] | (uint32_t)v[7] << 16);
    }
};

// Gradient of a 2x2 stride-2 transposed conv output, gathered at the input
// pixel's four children: k = (i * 2 + j) * C + c, t is the high-resolution tensor.
struct OpUpGather {
    Tens t; int64_t M; int K; int Hl, Wl;
    __device__ RowCtx prep(int64_t m) const {
        RowCtx rc; rc.ok = m < M; rc.pix = 0; rc.y = rc.x = 0;
        if (rc.ok) {
            int b; pixel_of(m, Hl, Wl, b, rc.y, rc.x);
            rc.pix = ((int64_t)b * t.H + 2 * rc.y) * t.W + 2 * rc.x;
        }
        return rc;
    }
    __device__ uint4 load(const RowCtx& rc, int k) const {
        if (!rc.ok || k >= K) return make_uint4(0, 0, 0, 0);
        const int ij = k / t.C, c = k - ij * t.C;
        const int64_t q = rc.pix + (int64_t)(ij >> 1) * t.W + (ij & 1);
        return *(const uint4*)(t.p + q * t.ld + t.off + c);
    }
};

// Plain row-major matrix: A[m][k] = p[m * ld + off + k].
struct OpPlain {
    const uint16_t* p; int64_t M; int K; int ld, off;
    __device__ RowCtx prep(int64_t m) const { RowCtx rc; rc.ok = m < M; rc.pix = m; rc.y = rc.x = 0; return rc; }
    __device__ uint4 load(const RowCtx& rc, int k) const {
        if (!rc.ok || k >= K) return make_uint4(0, 0, 0, 0);
        return *(const uint4*)(p + rc.pix * ld + off + k);
    }
};

// ---------------------------------------------------------------------------
// K-major operand policies (weight gradients, K = pixels): load_t(r0, k) gives
// rows r0..r0+7 at column k (zero outside).
// ---------------------------------------------------------------------------
// rows = channels of t, k = pixel.
struct OpChanT {
    Tens t; int R; int64_t K;
    __device__ uint4 load_t(int r0, int64_t k) const {
        if (r0 >= R || k >= K) return make_uint4(0, 0, 0, 0);
        return *(const uint4*)(t.p + k * t.ld + t.off + r0);
    }
};

// rows = (tap, c) of the 3x3 neighbourhood, k = output pixel.
struct OpIm2colT {
    Tens t; int R; int64_t K;
    __device__ uint4 load_t(int r0, int64_t k) const {
        if (r0 >= R || k >= K) return make_uint4(0, 0, 0, 0);
        const int tap = r0 / t.C, c = r0 - tap * t.C;
        int b, y, x;
        pixel_of(k, t.H, t.W, b, y, x);
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        if (y + dy < 0 || y + dy >= t.H || x + dx < 0 || x + dx >= t.W) return make_uint4(0, 0, 0, 0);
        return *(const uint4*)(t.p + (k + (int64_t)dy * t.W + dx) * t.ld + t.off + c);
    }
};

// rows = taps (< 9) of a single-channel input, k = output pixel.
struct OpIm2colTC1 {
    Tens t; int R; int64_t K;
    __device__ uint4 load_t(int r0, int64_t k) const {
        uint16_t v[8];
        int b = 0, y = 0, x = 0;
        if (k < K) pixel_of(k, t.H, t.W, b, y, x);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int tap = r0 + e;
            v[e] = 0;
            if (k < K && tap < 9) {
                const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                if (y + dy >= 0 && y + dy < t.H && x + dx >= 0 && x + dx < t.W)
                    v[e] = t.p[(k + (int64_t)dy * t.W + dx) * t.ld + t.off];
            }
        }
        return make_uint4(v[0] | (uint32_t)v[1] << 16, v[2] | (uint32_t)v[3] << 16, v[4] | (uint32_t)v[5] << 16,
                          v[6] | (uint32_t)v[7] << 16);
    }
};

// rows = channels of the high-resolution tensor t at child (i, j) of low-res pixel k.
struct OpUpChildT {
    Tens t; int R; int64_t K; int Hl, Wl, ij;
    __device__ uint4 load_t(int r0, int64_t k) const {
        if (r0 >= R || k >= K) return make_uint4(0, 0, 0, 0);
        int b, y, x;
        pixel_of(k, Hl, Wl, b, y, x);
        const int64_t q = ((int64_t)b * t.H + 2 * y + (ij >> 1)) * t.W + 2 * x + (ij & 1);
        return *(const uint4*)(t.p + q * t.ld + t.off + r0);
    }
};

// ---------------------------------------------------------------------------
// Epilogues: store(m, n, acc) for in-range elements.
// ---------------------------------------------------------------------------
// BF16 activation out[m * ld + off + n] = act(acc + bias[n]) (x mask, optional).
struct EpAct {
    static constexpr bool kStaged = true;
    uint16_t* p; int ld, off; const float* bias; int relu;
    const uint16_t* mask; int mld, moff;      // gradient through a ReLU: keep where mask > 0
    __device__ float act(int64_t, int n, float v) const {
        if (bias) v += bias[n];
        return relu ? fmaxf(v, 0.0f) : v;
    }
    __device__ void store(int64_t m, int n, float v) const {
        v = act(m, n, v);
        if (mask && !(bf2f(mask[m * mld + moff + n]) > 0.0f)) v = 0.0f;
        p[m * ld + off + n] = f2bf(v);
    }
    // columns n .. n+7 of row m, already activated, as 8 BF16
    __device__ void store8(int64_t m, int n, uint4 v) const {
        if (mask) {
            const uint4 k = *(const uint4*)(mask + m * mld + moff + n);
            const uint32_t kw[4] = {k.x, k.y, k.z, k.w};
            uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t lo = bf2f((uint16_t)(kw[e] & 0xFFFF)) > 0.0f ? 0x0000FFFFu : 0u;
                const uint32_t hi = bf2f((uint16_t)(kw[e] >> 16)) > 0.0f ? 0xFFFF0000u : 0u;
                vw[e] &= lo | hi;
            }
            v = make_uint4(vw[0], vw[1], vw[2], vw[3]);
        }
        *(uint4*)(p + m * ld + off + n) = v;
    }
};

// 2x2 stride-2 transposed conv output: n = (i * 2 + j) * C + c scatters to child (i, j).
struct EpUp {
    static constexpr bool kStaged = true;
    Tens t; int Hl, Wl; const float* bias;
    __device__ int64_t addr(int64_t m, int n) const {
        const int ij = n / t.C, c = n - ij * t.C;
        int b, y, x;
        pixel_of(m, Hl, Wl, b, y, x);
        const int64_t q = ((int64_t)b * t.H + 2 * y + (ij >> 1)) * t.W + 2 * x + (ij & 1);
        return q * t.ld + t.off + c;
    }
    __device__ float act(int64_t, int n, float v) const { return v + bias[n % t.C]; }
    __device__ void store(int64_t m, int n, float v) const { t.p[addr(m, n)] = f2bf(act(m, n, v)); }
    __device__ void store8(int64_t m, int n, uint4 v) const { *(uint4*)(t.p + addr(m, n)) = v; }
};

// FP32 split-K partial: part[z][m][n], z = the workgroup's K split.
struct EpPartial {
    static constexpr bool kStaged = false;
    float* p; int N; int64_t zstride;
    __device__ void store(int64_t m, int n, float v) const { p[blockIdx.z * zstride + m * N + n] = v; }
};

// ---------------------------------------------------------------------------
// The GEMM.  BM, BN in {32, 64, 128}; each wave owns (BM/2) x (BN/2) as
// (BM/32) x (BN/32) 16x16 MFMA tiles.  Operand A is row-major (RowOp) or
// K-major (AT = true), B likewise.  K range of this workgroup:
// [blockIdx.z * kchunk, min(K, (blockIdx.z + 1) * kchunk)).
// ---------------------------------------------------------------------------
template <int ROWS, class Op>
__device__ inline void stage_rows_fetch(const Op& op, const RowCtx* rc, int64_t k0, int64_t kend, uint4* reg) {
#pragma unroll
    for (int q = 0; q < (ROWS * 4 + NT - 1) / NT; ++q) {
        const int c = threadIdx.x + q * NT;
        const int kk = (c & 3) * 8;
        reg[q] = (c < ROWS * 4 && k0 + kk < kend) ? op.load(rc[q], (int)(k0 + kk)) : make_uint4(0, 0, 0, 0);
    }
}

template <int ROWS>
__device__ inline void stage_rows_store(uint16_t* lds, const uint4* reg) {
#pragma unroll
    for (int q = 0; q < (ROWS * 4 + NT - 1) / NT; ++q) {
        const int c = threadIdx.x + q * NT;
        if (c < ROWS * 4) *(uint4*)(lds + (c >> 2) * BKP + (c & 3) * 8) = reg[q];
    }
}

// K-major: chunk c covers rows 8 * (c % (ROWS/8)) .. +7 at column c / (ROWS/8).
template <int ROWS, class Op>
__device__ inline void stage_cols_fetch(const Op& op, int r_base, int64_t k0, int64_t kend, uint4* reg) {
#pragma unroll
    for (int q = 0; q < (ROWS * 4 + NT - 1) / NT; ++q) {
        const int c = threadIdx.x + q * NT;
        const int rg = c % (ROWS / 8), kk = c / (ROWS / 8);
        reg[q] = (c < ROWS * 4 && k0 + kk < kend) ? op.load_t(r_base + rg * 8, k0 + kk) : make_uint4(0, 0, 0, 0);
    }
}

// K-major tiles are kept pixel-major in LDS ([BK][ROWS + 8]): each fetched
// 16-byte chunk (8 rows at one k) is one 16-byte LDS write, and the MFMA
// fragment (8 consecutive k of one row) is gathered at read time, where it is
// reused across the wave's tiles.
template <int ROWS>
__device__ inline void stage_cols_store(uint16_t* lds, const uint4* reg) {
    constexpr int KP = ROWS + 8;
#pragma unroll
    for (int q = 0; q < (ROWS * 4 + NT - 1) / NT; ++q) {
        const int c = threadIdx.x + q * NT;
        if (c < ROWS * 4) {
            const int rg = c % (ROWS / 8), kk = c / (ROWS / 8);
            *(uint4*)(lds + kk * KP + rg * 8) = reg[q];
        }
    }
}

template <int ROWS>
__device__ inline bf16x8 frag_kmajor(const uint16_t* lds, int row, int g) {
    constexpr int KP = ROWS + 8;
    const uint16_t* p = lds + (8 * g) * KP + row;
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = (uint32_t)p[(2 * e) * KP] | ((uint32_t)p[(2 * e + 1) * KP] << 16);
    bf16x8 v;
    __builtin_memcpy(&v, w, sizeof(v));
    return v;
}

// Epilogue through LDS: the activated tile is staged as BF16 ([BM][BN + 8]) so
// that every thread writes whole 16-byte rows of 8 channels.  Needs N % 8 == 0
// and 16-byte aligned rows in the destination.
template <int BM, int BN, class EP, int TM, int TN>
__device__ inline void staged_epilogue(const EP& ep, const f32x4 (&acc)[TM][TN], uint16_t* stage, int64_t m0, int n0,
                                       int64_t M, int N, int wm, int wn, int g, int r16) {
    constexpr int SP = BN + 8;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rm = wm * (BM / 2) + i * 16 + g * 4 + e, rn = wn * (BN / 2) + j * 16 + r16;
                const int n = n0 + rn;
                stage[rm * SP + rn] = f2bf(n < N ? ep.act(m0 + rm, n, acc[i][j][e]) : 0.0f);
            }
    __syncthreads();
    for (int c = threadIdx.x; c < BM * (BN / 8); c += NT) {
        const int rm = c / (BN / 8), rn = (c % (BN / 8)) * 8;
        const int64_t m = m0 + rm;
        if (m < M && n0 + rn < N) ep.store8(m, n0 + rn, *(const uint4*)(stage + rm * SP + rn));
    }
}

template <int BM, int BN, class OA, bool AT, class OB, bool BT, class EP>
__global__ void __launch_bounds__(NT) k_gemm(OA oa, OB ob, EP ep, int64_t M, int N, int64_t K, int64_t kchunk) {
    constexpr int TM = BM / 32, TN = BN / 32;
    constexpr int CA = (BM * 4 + NT - 1) / NT, CB = (BN * 4 + NT - 1) / NT;
    // operand tiles (double-buffered); reused as the epilogue's staging tile
    __shared__ __attribute__((aligned(16))) uint16_t s_buf[2 * (BM + BN) * BKP];
    static_assert(BM * (BN + 8) <= 2 * (BM + BN) * BKP, "staging tile exceeds the operand buffers");
    uint16_t(*sA)[BM * BKP] = reinterpret_cast<uint16_t(*)[BM * BKP]>(s_buf);
    uint16_t(*sB)[BN * BKP] = reinterpret_cast<uint16_t(*)[BN * BKP]>(s_buf + 2 * BM * BKP);

    const int64_t m0 = (int64_t)blockIdx.x * BM;
    const int n0 = blockIdx.y * BN;
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    RowCtx rca[CA], rcb[CB];
    if constexpr (!AT) {
#pragma unroll
        for (int q = 0; q < CA; ++q) rca[q] = oa.prep(m0 + ((threadIdx.x + q * NT) >> 2));
    }
    if constexpr (!BT) {
#pragma unroll
        for (int q = 0; q < CB; ++q) rcb[q] = ob.prep((int64_t)n0 + ((threadIdx.x + q * NT) >> 2));
    }

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    uint4 ra[CA], rb[CB];
    auto fetch = [&](int64_t k0) {
        if constexpr (AT) stage_cols_fetch<BM>(oa, (int)m0, k0, ke, ra);
        else stage_rows_fetch<BM>(oa, rca, k0, ke, ra);
        if constexpr (BT) stage_cols_fetch<BN>(ob, n0, k0, ke, rb);
        else stage_rows_fetch<BN>(ob, rcb, k0, ke, rb);
    };
    auto put = [&](int buf) {
        if constexpr (AT) stage_cols_store<BM>(sA[buf], ra);
        else stage_rows_store<BM>(sA[buf], ra);
        if constexpr (BT) stage_cols_store<BN>(sB[buf], rb);
        else stage_rows_store<BN>(sB[buf], rb);
    };

    const int nsteps = ke > kb ? (int)((ke - kb + BK - 1) / BK) : 0;
    if (nsteps > 0) {
        fetch(kb);
        put(0);
    }
    __syncthreads();
    const int g = lane >> 4, r16 = lane & 15;
    for (int s = 0; s < nsteps; ++s) {
        const int buf = s & 1;
        if (s + 1 < nsteps) fetch(kb + (int64_t)(s + 1) * BK);
        bf16x8 fa[TM], fb[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if constexpr (AT) fa[i] = frag_kmajor<BM>(sA[buf], wm * (BM / 2) + i * 16 + r16, g);
            else fa[i] = *(const bf16x8*)(sA[buf] + (wm * (BM / 2) + i * 16 + r16) * BKP + g * 8);
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            if constexpr (BT) fb[j] = frag_kmajor<BN>(sB[buf], wn * (BN / 2) + j * 16 + r16, g);
            else fb[j] = *(const bf16x8*)(sB[buf] + (wn * (BN / 2) + j * 16 + r16) * BKP + g * 8);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        if (s + 1 < nsteps) put(buf ^ 1);
        __syncthreads();
    }
    // D layout: lane holds rows 4 * (lane / 16) + e of column lane % 16.
    if constexpr (EP::kStaged) {
        if (N % 8 == 0) {            // uniform: the loop above ended with a barrier
            staged_epilogue<BM, BN>(ep, acc, s_buf, m0, n0, M, N, wm, wn, g, r16);
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t m = m0 + wm * (BM / 2) + i * 16 + g * 4 + e;
                const int n = n0 + wn * (BN / 2) + j * 16 + r16;
                if (m < M && n < N) ep.store(m, n, acc[i][j][e]);
            }
}

template <int BM, int BN, class OA, bool AT, class OB, bool BT, class EP>
hipError_t gemm(const OA& oa, const OB& ob, const EP& ep, int64_t M, int N, int64_t K, int splits,
                int64_t kchunk, hipStream_t st) {
    const dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN), (unsigned)splits);
    hipLaunchKernelGGL((k_gemm<BM, BN, OA, AT, OB, BT, EP>), grid, dim3(NT), 0, st, oa, ob, ep, M, N, K, kchunk);
    return hipGetLastError();
}

// Tile width by the output-channel count.
template <class OA, class OB, class EP>
hipError_t gemm_rows(const OA& oa, const OB& ob, const EP& ep, int64_t M, int N, int64_t K, hipStream_t st) {
    if (N <= 32) return gemm<128, 32, OA, false, OB, false, EP>(oa, ob, ep, M, N, K, 1, K, st);
    if (N <= 64) return gemm<128, 64, OA, false, OB, false, EP>(oa, ob, ep, M, N, K, 1, K, st);
    return gemm<128, 128, OA, false, OB, false, EP>(oa, ob, ep, M, N, K, 1, K, st);
}

// Split-K weight-gradient GEMM into FP32 partials [splits][M][N]; returns splits.
template <class OA, class OB>
hipError_t gemm_wgrad(const OA& oa, const OB& ob, float* part, int M, int N, int64_t K, int max_splits,
                      int* splits_out, hipStream_t st) {
    const int bm = M <= 32 ? 32 : (M <= 64 ? 64 : 128);
    const int bn = N <= 32 ? 32 : (N <= 64 ? 64 : 128);
    const int64_t tiles = (int64_t)((M + bm - 1) / bm) * ((N + bn - 1) / bn);
    int64_t splits = (1024 + tiles - 1) / tiles;
    const int64_t max_by_k = (K + 4 * BK - 1) / (4 * BK);
    if (splits > max_by_k) splits = max_by_k;
    if (splits > max_splits) splits = max_splits;
    if (splits < 1) splits = 1;
    int64_t kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + BK - 1) / BK * BK;
    splits = (K + kchunk - 1) / kchunk;
    *splits_out = (int)splits;
    EpPartial ep{part, N, (int64_t)M * N};
    const dim3 grid((unsigned)((M + bm - 1) / bm), (unsigned)((N + bn - 1) / bn), (unsigned)splits);
#define BDC_WG(BMv, BNv) \
    if (bm == BMv && bn == BNv) { \
        hipLaunchKernelGGL((k_gemm<BMv, BNv, OA, true, OB, true, EpPartial>), grid, dim3(NT), 0, st, oa, ob, ep, \
                           (int64_t)M, N, K, kchunk); \
        return hipGetLastError(); }
    BDC_WG(32, 32) BDC_WG(32, 64) BDC_WG(32, 128)
    BDC_WG(64, 32) BDC_WG(64, 64) BDC_WG(64, 128)
    BDC_WG(128, 32) BDC_WG(128, 64) BDC_WG(128, 128)
#undef BDC_WG
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// 3x3 convolution with the input tile staged once per 32-channel slab.  An
// output tile of TH x TW pixels (128) x BN channels; for each slab of 32 input
// channels the (TH + 2) x (TW + 2) halo is loaded into LDS (zero outside the
// image, pixel pitch 40 elements: the 16 pixels one MFMA row-group reads fall
// in distinct banks), then the nine taps read their A fragments from it and
// their B fragments (weights, [c_out][tap][c_in]) straight from the L2.
// Every input pixel is read once per slab instead of once per tap.
// ---------------------------------------------------------------------------
constexpr int HALO_PP = 40;        // LDS elements per halo pixel (32 channels + pad)

// ONE: a single 32-channel slab (C = 32), whose halo needs no second buffer,
// so the workgroup holds half the LDS and more of them fit on a CU.
template <int BN, int TW, class EP, bool ONE>
__global__ void __launch_bounds__(NT) k_conv3_halo(Tens x, const uint16_t* wf, int K, EP ep, int N) {
    constexpr int TH = 128 / TW, HW = TW + 2, HH = TH + 2;
    constexpr int TM = 4, TN = BN / 32;
    constexpr int HALO = HH * HW * HALO_PP;
    constexpr int STAGE = 128 * (BN + 8);
    constexpr int NBUF = ONE ? 1 : 2;
    __shared__ __attribute__((aligned(16))) uint16_t s_buf[(NBUF * HALO > STAGE) ? NBUF * HALO : STAGE];
    const int tiles_x = x.W / TW, tiles_y = x.H / TH;
    const int tx = blockIdx.x % tiles_x, rest = blockIdx.x / tiles_x;
    const int ty = rest % tiles_y, b = rest / tiles_y;
    const int y0 = ty * TH, x0 = tx * TW;
    const int n0 = blockIdx.y * BN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int g = lane >> 4, r16 = lane & 15;
    const int C = x.C;

    // a slab's halo in two steps: every load of this thread issued into
    // registers first, then the LDS stores, so the loads are in flight
    // together (and, for the next slab, during this slab's taps)
    constexpr int NCH = HH * HW * 4, NIT = (NCH + NT - 1) / NT;
    uint4 hv[NIT];
    auto halo_issue = [&](int c0) {
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int c = threadIdx.x + k * NT;
            const int pix = c >> 2, q = c & 3;
            const int hy = pix / HW, hx = pix - hy * HW;
            const int yy = y0 + hy - 1, xx = x0 + hx - 1;
            hv[k] = make_uint4(0, 0, 0, 0);
            if (c < NCH && yy >= 0 && yy < x.H && xx >= 0 && xx < x.W)
                hv[k] = *(const uint4*)(x.p + (((int64_t)b * x.H + yy) * x.W + xx) * x.ld + x.off + c0 + q * 8);
        }
    };
    auto halo_commit = [&](uint16_t* h) {
#pragma unroll
        for (int k = 0; k < NIT; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c < NCH) *(uint4*)(h + (c >> 2) * HALO_PP + (c & 3) * 8) = hv[k];
        }
    };

    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    const int nslab = ONE ? 1 : C / 32;
    halo_issue(0);
    halo_commit(s_buf);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        uint16_t* h = s_buf + (sl & 1) * HALO;
        if (sl + 1 < nslab) halo_issue((sl + 1) * 32);
#pragma unroll 1
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3, dx = t % 3;        // halo offsets of this tap
            bf16x8 fa[TM], fb[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = n0 + wn * (BN / 2) + j * 16 + r16;
                fb[j] = n < N ? *(const bf16x8*)(wf + (int64_t)n * K + t * C + sl * 32 + g * 8) : bf16x8{};
            }
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int r = wm * 64 + i * 16 + r16;                  // output pixel in the tile
                const int py = r / TW, px = r - (r / TW) * TW;
                fa[i] = *(const bf16x8*)(h + ((py + dy) * HW + px + dx) * HALO_PP + g * 8);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        if (sl + 1 < nslab) halo_commit(s_buf + ((sl + 1) & 1) * HALO);
        __syncthreads();
    }
    // output rows: tile pixel r -> image pixel (b, y0 + r / TW, x0 + r % TW)
    struct EpTile {
        const EP& e; int b, y0, x0, H, W;
        __device__ int64_t pix(int r) const {
            return ((int64_t)b * H + y0 + r / TW) * W + x0 + r % TW;
        }
        __device__ float act(int64_t r, int n, float v) const { return e.act(pix((int)r), n, v); }
        __device__ void store8(int64_t r, int n, uint4 v) const { e.store8(pix((int)r), n, v); }
    } et{ep, b, y0, x0, x.H, x.W};
    staged_epilogue<128, BN>(et, acc, s_buf, 0, n0, 128, N, wm, wn, g, r16);
}

template <int BN, class EP>
hipError_t conv_halo_bn(const Tens& x, const uint16_t* wf, int K, const EP& ep, int N, int64_t P, hipStream_t st) {
    const int TW = x.W % 32 == 0 ? 32 : (x.W % 16 == 0 ? 16 : 8);
    const int TH = 128 / TW;
    const unsigned tiles = (unsigned)((int64_t)(x.W / TW) * (x.H / TH) * (P / ((int64_t)x.H * x.W)));
    const dim3 grid(tiles, (unsigned)((N + BN - 1) / BN));
    if (x.C == 32) {
        if (TW == 32) hipLaunchKernelGGL((k_conv3_halo<BN, 32, EP, true>), grid, dim3(NT), 0, st, x, wf, K, ep, N);
        else if (TW == 16) hipLaunchKernelGGL((k_conv3_halo<BN, 16, EP, true>), grid, dim3(NT), 0, st, x, wf, K, ep, N);
        else hipLaunchKernelGGL((k_conv3_halo<BN, 8, EP, true>), grid, dim3(NT), 0, st, x, wf, K, ep, N);
    } else {
        if (TW == 32) hipLaunchKernelGGL((k_conv3_halo<BN, 32, EP, false>), grid, dim3(NT), 0, st, x, wf, K, ep, N);
        else if (TW == 16) hipLaunchKernelGGL((k_conv3_halo<BN, 16, EP, false>), grid, dim3(NT), 0, st, x, wf, K, ep, N);
        else hipLaunchKernelGGL((k_conv3_halo<BN, 8, EP, false>), grid, dim3(NT), 0, st, x, wf, K, ep, N);
    }
    return hipGetLastError();
}

// Whether the halo kernel covers this input: 32-channel slabs, an output
// channel count that is a multiple of 32, tile rows that divide the image.
inline bool halo_ok(const Tens& x, int N) {
    if (x.C % 32 != 0 || N % 32 != 0 || x.ld % 8 != 0 || x.off % 8 != 0) return false;
    const int TW = x.W % 32 == 0 ? 32 : (x.W % 16 == 0 ? 16 : (x.W % 8 == 0 ? 8 : 0));
    return TW != 0 && x.H % (128 / TW) == 0;
}

template <class EP>
hipError_t conv_halo(const Tens& x, const uint16_t* wf, int K, const EP& ep, int N, int64_t P, hipStream_t st) {
    if (N <= 32) return conv_halo_bn<32>(x, wf, K, ep, N, P, st);
    if (N <= 64) return conv_halo_bn<64>(x, wf, K, ep, N, P, st);
    return conv_halo_bn<128>(x, wf, K, ep, N, P, st);
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
// Sum of split-K partials into FP32 gradient entries: out[base + m * ms + n * ns] = sum_z part[z][m][n].
// A workgroup takes 64 consecutive entries; its four waves sum every fourth
// split each (loads of a wave coalesced along the entries, four independent
// accumulators per thread), then combine.
constexpr int RED_ENTRIES = 64;
__global__ void __launch_bounds__(256) k_reduce_partials(const float* part, int splits, int M, int N, float* out,
                                                         int64_t ms, int64_t ns) {
    __shared__ float s_sum[4][RED_ENTRIES];
    const int o = threadIdx.x & (RED_ENTRIES - 1), ph = threadIdx.x / RED_ENTRIES;
    const int64_t MN = (int64_t)M * N;
    const int64_t i = (int64_t)blockIdx.x * RED_ENTRIES + o;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;    // four independent chains of loads
    if (i < MN) {
        int z = ph;
        for (; z + 12 < splits; z += 16) {
            s0 += part[(int64_t)z * MN + i];
            s1 += part[(int64_t)(z + 4) * MN + i];
            s2 += part[(int64_t)(z + 8) * MN + i];
            s3 += part[(int64_t)(z + 12) * MN + i];
        }
        for (; z < splits; z += 4) s0 += part[(int64_t)z * MN + i];
    }
    s_sum[ph][o] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (ph == 0 && i < MN) {
        const int m = (int)(i / N), n = (int)(i - (int64_t)m * N);
        out[m * ms + n * ns] = (s_sum[0][o] + s_sum[1][o]) + (s_sum[2][o] + s_sum[3][o]);
    }
}

// Per-channel column sums of a BF16 slice over P pixels -> partial[wg][C].
__global__ void k_colsum(Tens t, int64_t P, int64_t per_wg, float* part) {
    __shared__ float s_acc[NT];
    const int C = t.C;
    const int lanes_per_c = NT / C;               // C divides NT (C <= 256, power of two)
    const int c = threadIdx.x % C, sub = threadIdx.x / C;
    const int64_t p0 = (int64_t)blockIdx.x * per_wg;
    const int64_t p1 = p0 + per_wg < P ? p0 + per_wg : P;
    float s = 0.0f;
    for (int64_t p = p0 + sub; p < p1; p += lanes_per_c) s += bf2f(t.p[p * t.ld + t.off + c]);
    s_acc[threadIdx.x] = s;
    __syncthreads();
    if (sub == 0) {
        float tot = 0.0f;
        for (int q = 0; q < lanes_per_c; ++q) tot += s_acc[q * C + c];
        part[(int64_t)blockIdx.x * C + c] = tot;
    }
}

// out[c] = sum_w part[w][c]: one workgroup per column, fixed-order tree.
__global__ void __launch_bounds__(NT) k_sum_rows(const float* part, int nw, int C, float* out) {
    __shared__ float s_r[NT];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int w = threadIdx.x; w < nw; w += NT) s += part[(int64_t)w * C + c];
    s_r[threadIdx.x] = s;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) s_r[threadIdx.x] += s_r[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = s_r[0];
}

// Weight gradient of the single-channel input layer: dW[co][tap] =
// sum_p g[p][co] x[p + off(tap)], nine sums per output channel; a plain
// reduction (0.3 GFLOP at 8 x 256^2), one partial row [co * 9 + tap] per workgroup.
__global__ void __launch_bounds__(NT) k_wgrad_c1(Tens x, Tens g, int64_t P, int64_t per_wg, float* part) {
    __shared__ float s_p[NT * 9];
    const int C = g.C;                           // divides NT
    const int co = threadIdx.x % C, sub = threadIdx.x / C, nsub = NT / C;
    const int64_t p0 = (int64_t)blockIdx.x * per_wg;
    const int64_t p1 = p0 + per_wg < P ? p0 + per_wg : P;
    float acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.0f;
    for (int64_t p = p0 + sub; p < p1; p += nsub) {
        const float gv = bf2f(g.p[p * g.ld + g.off + co]);
        int b, y, xx;
        pixel_of(p, x.H, x.W, b, y, xx);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            if (y + dy >= 0 && y + dy < x.H && xx + dx >= 0 && xx + dx < x.W)
                acc[t] = fmaf(gv, bf2f(x.p[(p + (int64_t)dy * x.W + dx) * x.ld + x.off]), acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) s_p[t * NT + threadIdx.x] = acc[t];
    __syncthreads();
    for (int q = threadIdx.x; q < 9 * C; q += NT) {
        const int c = q / 9, t = q % 9;
        float tot = 0.0f;
        for (int u = 0; u < nsub; ++u) tot += s_p[t * NT + u * C + c];
        part[(int64_t)blockIdx.x * 9 * C + q] = tot;
    }
}

// 2x2 max pool of a slice: out at (H/2, W/2).
__global__ void k_maxpool(Tens in, Tens out, int64_t P_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P_out * out.C) return;
    const int64_t p = i / out.C;
    const int c = (int)(i - p * out.C);
    int b, y, x;
    pixel_of(p, out.H, out.W, b, y, x);
    const int64_t q = ((int64_t)b * in.H + 2 * y) * in.W + 2 * x;
    float m = bf2f(in.p[q * in.ld + in.off + c]);
    m = fmaxf(m, bf2f(in.p[(q + 1) * in.ld + in.off + c]));
    m = fmaxf(m, bf2f(in.p[(q + in.W) * in.ld + in.off + c]));
    m = fmaxf(m, bf2f(in.p[(q + in.W + 1) * in.ld + in.off + c]));
    out.p[p * out.ld + out.off + c] = f2bf(m);
}

// Pool backward into the pooled tensor's gradient slice, which already holds the
// skip path's contribution; the sum is then taken through the ReLU that made
// the pooled input: gin = (gin + [first argmax] gout) * [in > 0].
__global__ void k_maxpool_bwd(Tens in, Tens gin, Tens gout, int64_t P_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P_out * gout.C) return;
    const int64_t p = i / gout.C;
    const int c = (int)(i - p * gout.C);
    int b, y, x;
    pixel_of(p, gout.H, gout.W, b, y, x);
    const int64_t q0 = ((int64_t)b * in.H + 2 * y) * in.W + 2 * x;
    const int64_t qs[4] = {q0, q0 + 1, q0 + in.W, q0 + in.W + 1};
    float v[4];
    int am = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[e] = bf2f(in.p[qs[e] * in.ld + in.off + c]);
        if (v[e] > v[am]) am = e;
    }
    const float g = bf2f(gout.p[p * gout.ld + gout.off + c]);
    uint16_t* gp = gin.p;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t a = qs[e] * gin.ld + gin.off + c;
        float s = bf2f(gp[a]) + (e == am ? g : 0.0f);
        gp[a] = f2bf(v[e] > 0.0f ? s : 0.0f);
    }
}

// The same two passes eight channels at a time (C, ld and off multiples of 8:
// 16-byte loads and stores), with each channel's arithmetic and order as above.
__device__ inline uint32_t bf2_max4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    float lo = bf2f((uint16_t)a);
    lo = fmaxf(lo, bf2f((uint16_t)b));
    lo = fmaxf(lo, bf2f((uint16_t)c));
    lo = fmaxf(lo, bf2f((uint16_t)d));
    float hi = bf2f((uint16_t)(a >> 16));
    hi = fmaxf(hi, bf2f((uint16_t)(b >> 16)));
    hi = fmaxf(hi, bf2f((uint16_t)(c >> 16)));
    hi = fmaxf(hi, bf2f((uint16_t)(d >> 16)));
    return (uint32_t)f2bf(lo) | (uint32_t)f2bf(hi) << 16;
}

__global__ void k_maxpool8(Tens in, Tens out, int64_t P_out) {
    const int c8 = out.C >> 3;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P_out * c8) return;
    const int64_t p = i / c8;
    const int c = (int)(i - p * c8) * 8;
    int b, y, x;
    pixel_of(p, out.H, out.W, b, y, x);
    const int64_t q = ((int64_t)b * in.H + 2 * y) * in.W + 2 * x;
    const uint4 v0 = *(const uint4*)(in.p + q * in.ld + in.off + c);
    const uint4 v1 = *(const uint4*)(in.p + (q + 1) * in.ld + in.off + c);
    const uint4 v2 = *(const uint4*)(in.p + (q + in.W) * in.ld + in.off + c);
    const uint4 v3 = *(const uint4*)(in.p + (q + in.W + 1) * in.ld + in.off + c);
    *(uint4*)(out.p + p * out.ld + out.off + c) =
        make_uint4(bf2_max4(v0.x, v1.x, v2.x, v3.x), bf2_max4(v0.y, v1.y, v2.y, v3.y),
                   bf2_max4(v0.z, v1.z, v2.z, v3.z), bf2_max4(v0.w, v1.w, v2.w, v3.w));
}

__global__ void k_maxpool8_bwd(Tens in, Tens gin, Tens gout, int64_t P_out) {
    const int c8 = gout.C >> 3;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P_out * c8) return;
    const int64_t p = i / c8;
    const int c = (int)(i - p * c8) * 8;
    int b, y, x;
    pixel_of(p, gout.H, gout.W, b, y, x);
    const int64_t q0 = ((int64_t)b * in.H + 2 * y) * in.W + 2 * x;
    const int64_t qs[4] = {q0, q0 + 1, q0 + in.W, q0 + in.W + 1};
    uint32_t v[4][4], gi[4][4], go[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint4 a = *(const uint4*)(in.p + qs[e] * in.ld + in.off + c);
        const uint4 g = *(const uint4*)(gin.p + qs[e] * gin.ld + gin.off + c);
        v[e][0] = a.x; v[e][1] = a.y; v[e][2] = a.z; v[e][3] = a.w;
        gi[e][0] = g.x; gi[e][1] = g.y; gi[e][2] = g.z; gi[e][3] = g.w;
    }
    {
        const uint4 g = *(const uint4*)(gout.p + p * gout.ld + gout.off + c);
        go[0] = g.x; go[1] = g.y; go[2] = g.z; go[3] = g.w;
    }
    auto half = [](uint32_t w, int h) { return (uint16_t)(h ? w >> 16 : w & 0xFFFFu); };
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int wd = k >> 1, h = k & 1;
        int am = 0;
#pragma unroll
        for (int e = 1; e < 4; ++e)
            if (bf2f(half(v[e][wd], h)) > bf2f(half(v[am][wd], h))) am = e;
        const float g = bf2f(half(go[wd], h));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float sum = bf2f(half(gi[e][wd], h)) + (e == am ? g : 0.0f);
            const uint32_t r = f2bf(bf2f(half(v[e][wd], h)) > 0.0f ? sum : 0.0f);
            gi[e][wd] = h ? ((gi[e][wd] & 0xFFFFu) | r << 16) : ((gi[e][wd] & 0xFFFF0000u) | r);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
        *(uint4*)(gin.p + qs[e] * gin.ld + gin.off + c) = make_uint4(gi[e][0], gi[e][1], gi[e][2], gi[e][3]);
}

// 3x3 convolution of a single-channel input, eight output channels per thread
// (N, y.ld and y.off multiples of 8): the nine taps of one pixel against
// weights staged in LDS (wf [N][16], taps 0..8 = (dy + 1) * 3 + dx + 1), FP32
// accumulation, bias and ReLU as the GEMM epilogue, one 16-byte store.
constexpr int C1_MAXN = 256;
__global__ void __launch_bounds__(256) k_conv3_c1(Tens x, const uint16_t* wf, const float* bias, int relu, Tens y,
                                                  int64_t P) {
    __shared__ float s_w[C1_MAXN * 9];
    __shared__ float s_b[C1_MAXN];
    const int N = y.C;
    for (int q = threadIdx.x; q < N * 9; q += blockDim.x) s_w[q] = bf2f(wf[(q / 9) * 16 + q % 9]);
    for (int q = threadIdx.x; q < N; q += blockDim.x) s_b[q] = bias ? bias[q] : 0.0f;
    __syncthreads();
    const int n8 = N >> 3;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * n8) return;
    const int64_t p = i / n8;
    const int n0 = (int)(i - p * n8) * 8;
    int b, py, px;
    pixel_of(p, x.H, x.W, b, py, px);
    float in[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int dy = t / 3 - 1, dx = t % 3 - 1, yy = py + dy, xx = px + dx;
        in[t] = (yy >= 0 && yy < x.H && xx >= 0 && xx < x.W)
                    ? bf2f(x.p[(p + (int64_t)dy * x.W + dx) * x.ld + x.off]) : 0.0f;
    }
    uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float* w = s_w + (n0 + k) * 9;
        float a = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) a = fmaf(w[t], in[t], a);
        a += s_b[n0 + k];
        o[k >> 1] |= (uint32_t)f2bf(relu ? fmaxf(a, 0.0f) : a) << (16 * (k & 1));
    }
    *(uint4*)(y.p + p * y.ld + y.off + n0) = make_uint4(o[0], o[1], o[2], o[3]);
}

// FP32 [P] -> BF16 single-channel tensor.
__global__ void k_to_bf16(const float* x, int64_t n, uint16_t* y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// 1x1 head (C -> 2: mean and log-std of log rho) with the training loss
//   L = (1/P) sum_p [(m_p - y_p)^2 + (s_p - z_p)^2]
// and its gradient: dF (through the last ReLU) as BF16, and per-workgroup
// partials [wg][2C + 3] of dW [2][C], db [2] and the loss sum.
// target == nullptr: inference only.
template <int C>
__global__ void __launch_bounds__(128) k_head(Tens f, const float* w, const float* bias, int64_t P, float* out,
                                              const float* target, uint16_t* gf, float* part) {
    constexpr int RW = 2 * C + 3;
    __shared__ float s_h[128 * RW];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float m = 0.0f, s = 0.0f;
    float fv[C];
    const bool ok = p < P;
    if (ok) {
        m = bias[0];
        s = bias[1];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            fv[c] = bf2f(f.p[p * f.ld + f.off + c]);
            m = fmaf(w[c], fv[c], m);
            s = fmaf(w[C + c], fv[c], s);
        }
        out[2 * p] = m;
        out[2 * p + 1] = s;
    }
    if (!target) return;                       // uniform over the launch
    float* row = s_h + threadIdx.x * RW;
    if (ok) {
        const float em = m - target[2 * p], es = s - target[2 * p + 1];
        const float gm = 2.0f * em / (float)P, gs = 2.0f * es / (float)P;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float g = fmaf(gm, w[c], gs * w[C + c]);
            gf[p * f.ld + f.off + c] = f2bf(fv[c] > 0.0f ? g : 0.0f);
            row[c] = gm * fv[c];
            row[C + c] = gs * fv[c];
        }
        row[2 * C] = gm;
        row[2 * C + 1] = gs;
        row[2 * C + 2] = em * em + es * es;
    } else {
        for (int q = 0; q < RW; ++q) row[q] = 0.0f;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < RW; q += blockDim.x) {
        float tot = 0.0f;
        for (int t = 0; t < (int)blockDim.x; ++t) tot += s_h[t * RW + q];
        part[(int64_t)blockIdx.x * RW + q] = tot;
    }
}

// Adam with bias correction on FP32 master weights.
__global__ void k_adam(float* p, float* m1, float* m2, const float* g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// BF16 operand copies of one 3x3 layer's master weights W[co][tap][ci]:
//   fwd[co][kp], k = tap * ci_n + ci (zero-padded to kp);
//   dgrad[ci][tap' * co_n + co] = W[co][8 - tap'][ci] (null for the input layer).
__global__ void k_wconv3(const float* W, int co_n, int ci_n, int kp, uint16_t* fwd, uint16_t* dgrad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nf = (int64_t)co_n * kp;
    if (i < nf) {
        const int co = (int)(i / kp), k = (int)(i - (int64_t)co * kp);
        fwd[i] = k < 9 * ci_n ? f2bf(W[(int64_t)co * 9 * ci_n + k]) : (uint16_t)0;
    }
    if (dgrad && i < (int64_t)co_n * 9 * ci_n) {
        const int ci = (int)(i / (9 * co_n));
        const int r = (int)(i - (int64_t)ci * 9 * co_n);
        const int tp = r / co_n, co = r - tp * co_n;
        dgrad[i] = f2bf(W[((int64_t)co * 9 + (8 - tp)) * ci_n + ci]);
    }
}

// Transposed 2x2 layer, master Wt[ij][co][ci]: fwd = same order;
// dgrad[ci][ij * co_n + co].
__global__ void k_wup(const float* W, int co_n, int ci_n, uint16_t* fwd, uint16_t* dgrad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)4 * co_n * ci_n;
    if (i >= n) return;
    fwd[i] = f2bf(W[i]);
    const int ci = (int)(i / (4 * co_n));
    const int r = (int)(i - (int64_t)ci * 4 * co_n);          // ij * co_n + co
    dgrad[i] = f2bf(W[(int64_t)r * ci_n + ci]);
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
hipError_t conv3_fwd(const Tens& x, const uint16_t* wf, const float* bias, int relu, const Tens& y, int64_t P,
                     hipStream_t st) {
    EpAct ep{y.p, y.ld, y.off, bias, relu, nullptr, 0, 0};
    OpPlain ob{wf, (int64_t)y.C, 0, 0, 0};
    if (x.C == 1) {
        if (y.C % 8 == 0 && y.C <= C1_MAXN && y.ld % 8 == 0 && y.off % 8 == 0) {
            hipLaunchKernelGGL(k_conv3_c1, dim3(nblk(P * (y.C / 8))), dim3(256), 0, st, x, wf, bias, relu, y, P);
            return hipGetLastError();
        }
        ob.K = 16; ob.ld = 16;
        return gemm_rows(OpConv3C1{x, P}, ob, ep, P, y.C, 16, st);
    }
    const int K = 9 * x.C;
    if (halo_ok(x, y.C)) return conv_halo(x, wf, K, ep, y.C, P, st);
    ob.K = K; ob.ld = K;
    return gemm_rows(OpConv3{x, P, K}, ob, ep, P, y.C, K, st);
}

hipError_t conv3_dgrad(const Tens& g, const uint16_t* wd, const Tens& gx, const Tens* mask, int64_t P,
                       hipStream_t st) {
    const int K = 9 * g.C;
    EpAct ep{gx.p, gx.ld, gx.off, nullptr, 0, mask ? mask->p : nullptr,
             mask ? mask->ld : 0, mask ? mask->off : 0};
    if (halo_ok(g, gx.C)) return conv_halo(g, wd, K, ep, gx.C, P, st);
    OpPlain ob{wd, (int64_t)gx.C, K, K, 0};
    return gemm_rows(OpConv3{g, P, K}, ob, ep, P, gx.C, K, st);
}

hipError_t conv3_wgrad(const Tens& x, const Tens& g, float* part, int max_splits, float* dw, int64_t P,
                       hipStream_t st) {
    int splits = 1;
    hipError_t e;
    const int N = x.C == 1 ? 9 : 9 * x.C;
    if (x.C == 1) {
        int64_t per = (P + 1023) / 1024;
        if (per < 256) per = 256;
        const int nw = (int)((P + per - 1) / per);
        if ((int64_t)nw * 9 * g.C > PART_MAX) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_wgrad_c1, dim3(nw), dim3(NT), 0, st, x, g, P, per, part);
        hipLaunchKernelGGL(k_sum_rows, dim3(9 * g.C), dim3(NT), 0, st, part, nw, 9 * g.C, dw);
        return hipGetLastError();
    }
    e = gemm_wgrad(OpChanT{g, g.C, P}, OpIm2colT{x, N, P}, part, g.C, N, P, max_splits, &splits, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_partials, dim3(nblk((int64_t)g.C * N, RED_ENTRIES)), dim3(256), 0, st, part, splits,
                       g.C, N, dw,
                       (int64_t)N, (int64_t)1);
    return hipGetLastError();
}

hipError_t up_fwd(const Tens& x, const uint16_t* wf, const float* bias, const Tens& y, int64_t P_lo, int Hl, int Wl,
                  hipStream_t st) {
    EpUp ep{y, Hl, Wl, bias};
    OpPlain oa{x.p, P_lo, x.C, x.ld, x.off};
    OpPlain ob{wf, (int64_t)4 * y.C, x.C, x.C, 0};
    return gemm_rows(oa, ob, ep, P_lo, 4 * y.C, x.C, st);
}

hipError_t up_dgrad(const Tens& g, const uint16_t* wd, const Tens& gx, const Tens* mask, int64_t P_lo, int Hl,
                    int Wl, hipStream_t st) {
    const int K = 4 * g.C;
    EpAct ep{gx.p, gx.ld, gx.off, nullptr, 0, mask ? mask->p : nullptr,
             mask ? mask->ld : 0, mask ? mask->off : 0};
    OpPlain ob{wd, (int64_t)gx.C, K, K, 0};
    return gemm_rows(OpUpGather{g, P_lo, K, Hl, Wl}, ob, ep, P_lo, gx.C, K, st);
}

hipError_t up_wgrad(const Tens& x, const Tens& g, float* part, int max_splits, float* dw, int64_t P_lo, int Hl,
                    int Wl, hipStream_t st) {
    for (int ij = 0; ij < 4; ++ij) {
        int splits = 1;
        // C[m = ci][n = co] -> Wt[ij][co][ci]
        hipError_t e = gemm_wgrad(OpChanT{x, x.C, P_lo}, OpUpChildT{g, g.C, P_lo, Hl, Wl, ij}, part, x.C, g.C, P_lo,
                                  max_splits, &splits, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_reduce_partials, dim3(nblk((int64_t)x.C * g.C, RED_ENTRIES)), dim3(256), 0, st, part,
                           splits, x.C,
                           g.C, dw + (int64_t)ij * g.C * x.C, (int64_t)1, (int64_t)x.C);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t bias_grad(const Tens& g, int64_t P, float* part, int max_wg, float* db, hipStream_t st) {
    int64_t per = (P + max_wg - 1) / max_wg;
    if (per < 64) per = 64;
    const int nw = (int)((P + per - 1) / per);
    hipLaunchKernelGGL(k_colsum, dim3(nw), dim3(NT), 0, st, g, P, per, part);
    hipLaunchKernelGGL(k_sum_rows, dim3(g.C), dim3(NT), 0, st, part, nw, g.C, db);
    return hipGetLastError();
}

static bool vec8(const Tens& t) { return t.C % 8 == 0 && t.ld % 8 == 0 && t.off % 8 == 0; }

hipError_t maxpool(const Tens& in, const Tens& out, int64_t P_out, hipStream_t st) {
    if (vec8(in) && vec8(out) && in.C == out.C)
        hipLaunchKernelGGL(k_maxpool8, dim3(nblk(P_out * (out.C / 8))), dim3(256), 0, st, in, out, P_out);
    else
        hipLaunchKernelGGL(k_maxpool, dim3(nblk(P_out * out.C)), dim3(256), 0, st, in, out, P_out);
    return hipGetLastError();
}

hipError_t maxpool_bwd(const Tens& in, const Tens& gin, const Tens& gout, int64_t P_out, hipStream_t st) {
    if (vec8(in) && vec8(gin) && vec8(gout) && in.C == gout.C && gin.C == gout.C)
        hipLaunchKernelGGL(k_maxpool8_bwd, dim3(nblk(P_out * (gout.C / 8))), dim3(256), 0, st, in, gin, gout, P_out);
    else
        hipLaunchKernelGGL(k_maxpool_bwd, dim3(nblk(P_out * gout.C)), dim3(256), 0, st, in, gin, gout, P_out);
    return hipGetLastError();
}

hipError_t to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(256), 0, st, x, n, y);
    return hipGetLastError();
}

constexpr int HEAD_NT = 128;

int head_partial_rows(int64_t P) { return (int)((P + HEAD_NT - 1) / HEAD_NT); }

hipError_t head(const Tens& f, const float* w, const float* b, int64_t P, float* out, const float* target,
                uint16_t* gf, float* part, float* sums, hipStream_t st) {
    const int nw = head_partial_rows(P);
    switch (f.C) {
    case 8: hipLaunchKernelGGL(k_head<8>, dim3(nw), dim3(HEAD_NT), 0, st, f, w, b, P, out, target, gf, part); break;
    case 16: hipLaunchKernelGGL(k_head<16>, dim3(nw), dim3(HEAD_NT), 0, st, f, w, b, P, out, target, gf, part); break;
    case 32: hipLaunchKernelGGL(k_head<32>, dim3(nw), dim3(HEAD_NT), 0, st, f, w, b, P, out, target, gf, part); break;
    case 64: hipLaunchKernelGGL(k_head<64>, dim3(nw), dim3(HEAD_NT), 0, st, f, w, b, P, out, target, gf, part); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !target) return e;
    const int RW = 2 * f.C + 3;
    hipLaunchKernelGGL(k_sum_rows, dim3(RW), dim3(NT), 0, st, part, nw, RW, sums);
    return hipGetLastError();
}

hipError_t adam(float* p, float* m1, float* m2, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, st, p, m1, m2, g, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t weights_conv3(const float* W, int co_n, int ci_n, uint16_t* fwd, uint16_t* dgrad, hipStream_t st) {
    const int kp = ci_n == 1 ? 16 : 9 * ci_n;
    const int64_t n = (int64_t)co_n * (kp > 9 * ci_n ? kp : 9 * ci_n);
    hipLaunchKernelGGL(k_wconv3, dim3(nblk(n)), dim3(256), 0, st, W, co_n, ci_n, kp, fwd, dgrad);
    return hipGetLastError();
}

hipError_t weights_up(const float* W, int co_n, int ci_n, uint16_t* fwd, uint16_t* dgrad, hipStream_t st) {
    hipLaunchKernelGGL(k_wup, dim3(nblk((int64_t)4 * co_n * ci_n)), dim3(256), 0, st, W, co_n, ci_n, fwd, dgrad);
    return hipGetLastError();
}

// Plain GEMM C[M][N] = A[M][K] B[N][K]^T (BF16 in, FP32 out) -- exposed for tests of the MFMA tile.
struct EpF32 {
    static constexpr bool kStaged = false;
    float* p; int N;
    __device__ void store(int64_t m, int n, float v) const { p[m * N + n] = v; }
};

hipError_t gemm_nt(const uint16_t* a, const uint16_t* b, float* c, int64_t M, int N, int K, hipStream_t st) {
    return gemm_rows(OpPlain{a, M, K, K, 0}, OpPlain{b, (int64_t)N, K, K, 0}, EpF32{c, N}, M, N, K, st);
}

}  // namespace unet
}  // namespace bdc
