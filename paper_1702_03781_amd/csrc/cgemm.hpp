// Batched complex GEMM on the matrix cores (MFMA) for gfx950:
//   D = beta * C + alpha * A * B      (alpha, beta real; D may alias C)
// Column-major, interleaved complex (re, im), complex64 (T = float) or
// complex128 (T = double).  Used by the blocked LU (trailing and intra-panel
// updates), the triangular solves and the FP64 refinement residual.
//
// Complex as real MFMA.  With real index 2i (re) / 2i+1 (im) on rows and on
// the contraction index, a complex product C = A B is the real product
// C~ = A~ B~ with
//   A~[2i][2k] = a_re, A~[2i][2k+1] = -a_im, A~[2i+1][2k] = a_im, A~[2i+1][2k+1] = a_re,
//   B~[2k][j]  = b_re, B~[2k+1][j]  = b_im,   C~[2i][j] = c_re, C~[2i+1][j] = c_im.
// B~ and C~ are exactly the interleaved column-major storage viewed as real,
// and every A~ entry is a signed component of one stored complex number, so
// the operands go from LDS to the MFMA with a component select and a sign:
// 8 real flops per complex multiply-add, no extra traffic.
//
// Instruction: v_mfma_{f32,f64}_16x16x4 (16 real rows x 16 columns x 4 real
// k = 8 complex rows x 16 columns x 2 complex k).  Lane l feeds A~[l%16][l/16]
// and B~[l/16][l%16] and receives four entries of column l%16 of C~ (rows
// 4(l/16)+v for the f32 form, 4v+l/16 for the f64 form, v = 0..3).
//
// Tiling: 256 threads = 2 x 2 waves; workgroup tile BM complex rows x BN
// columns, K streamed in BK-wide complex chunks through double-buffered LDS
// (A chunk stored [k][row], B chunk [col][k] padded by one complex to spread
// banks).  Each wave owns (BM/2) x (BN/2): (BM/16) x (BN/32) MFMA blocks.
#pragma once

#include "common.hpp"
#include "prof.hpp"

namespace harp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// out_row(lane, v): real row (0..15) of accumulator element v of `lane`; the
// column is lane % 16.  The two instructions order their outputs differently.
template <> struct Mfma<float> {
    using acc_t = f32x4;
    using c_t = float2;
    __device__ static acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
    using acc_t = f64x4;
    using c_t = double2;
    __device__ static acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int out_row(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <typename T> struct GemmArgs {
    int M, N, K;                 // complex dimensions
    const T* A;                  // interleaved complex, column-major
    int64_t lda, sA;             // leading dimension / batch stride (complex elements)
    const T* B;
    int64_t ldb, sB;
    const T* C;                  // may be null when beta == 0
    int64_t ldc, sC;
    T* D;
    int64_t ldd, sD;
    T alpha, beta;
    const int32_t* active;       // optional [outer batch]: 0 skips that matrix
    // optional second batch level: grid z = outer * inner + i, operand X at
    // X + outer * sX + i * sX2 (e.g. several blocks of one matrix)
    int inner = 1;
    int64_t sA2 = 0, sB2 = 0, sC2 = 0, sD2 = 0;
};

template <typename T, int BM, int BN, int BK>
__global__ void __launch_bounds__(256) cgemm_kernel(GemmArgs<T> g) {
    using ct = typename Mfma<T>::c_t;
    using acc_t = typename Mfma<T>::acc_t;
    constexpr int RB = BM / 16;          // MFMA row blocks per wave (8 complex rows each)
    constexpr int CB = BN / 32;          // MFMA column blocks per wave (16 columns each)
    constexpr int A_PER_T = BM * BK / 256;
    constexpr int B_PER_T = BN * BK / 256;
    static_assert(BM % 16 == 0 && BN % 32 == 0 && BK % 2 == 0, "tile shape");
    static_assert(A_PER_T >= 1 && B_PER_T >= 1, "tile too small for 256 threads");

    const int bz = blockIdx.z / g.inner, bi = blockIdx.z % g.inner;
    if (g.active && g.active[bz] == 0) return;
    const int tiles_m = (g.M + BM - 1) / BM;
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int row0 = tm * BM, col0 = tn * BN;

    const ct* A = reinterpret_cast<const ct*>(g.A) + size_t(bz) * g.sA + size_t(bi) * g.sA2;
    const ct* B = reinterpret_cast<const ct*>(g.B) + size_t(bz) * g.sB + size_t(bi) * g.sB2;

    __shared__ ct As[2][BK][BM];
    __shared__ ct Bs[2][BN][BK + 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave & 1) * (BM / 2);    // wave's complex-row offset in the tile
    const int wc = (wave >> 1) * (BN / 2);   // wave's column offset in the tile

    // global -> register staging
    ct ra[A_PER_T], rb[B_PER_T];
    // A chunk: thread owns k = tid / (BM / A_PER_T), rows (tid % (BM / A_PER_T)) * A_PER_T + e
    constexpr int A_ROW_GROUPS = BM / A_PER_T;
    const int a_k = tid / A_ROW_GROUPS, a_r = (tid % A_ROW_GROUPS) * A_PER_T;
    // B chunk: thread owns column tid / (BK / B_PER_T), k (tid % (BK / B_PER_T)) * B_PER_T + e
    constexpr int B_K_GROUPS = BK / B_PER_T;
    const int b_c = tid / B_K_GROUPS, b_k = (tid % B_K_GROUPS) * B_PER_T;

    auto load_chunk = [&](int k0) {
        const int ka = k0 + a_k;
#pragma unroll
        for (int e = 0; e < A_PER_T; ++e) {
            const int r = row0 + a_r + e;
            ra[e] = (r < g.M && ka < g.K) ? A[size_t(ka) * g.lda + r] : ct{T(0), T(0)};
        }
        const int cb = col0 + b_c;
#pragma unroll
        for (int e = 0; e < B_PER_T; ++e) {
            const int kb = k0 + b_k + e;
            rb[e] = (cb < g.N && kb < g.K) ? B[size_t(cb) * g.ldb + kb] : ct{T(0), T(0)};
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int e = 0; e < A_PER_T; ++e) As[buf][a_k][a_r + e] = ra[e];
#pragma unroll
        for (int e = 0; e < B_PER_T; ++e) Bs[buf][b_c][b_k + e] = rb[e];
    };

    // accumulators start at beta * C (read before the K loop so its latency
    // overlaps the first A/B chunk); alpha is folded into the A operand
    const int b_col = lane & 15;
    const int M2 = 2 * g.M;
    acc_t acc[RB][CB];
    {
        const T* Cr = g.C ? g.C + 2 * (size_t(bz) * g.sC + size_t(bi) * g.sC2) : nullptr;
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int col = col0 + wc + j * 16 + b_col;
                const int rbase = 2 * (row0 + wr + i * 8);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = rbase + Mfma<T>::out_row(lane, v);
                    acc[i][j][v] = (g.beta != T(0) && col < g.N && rr < M2)
                                       ? g.beta * Cr[2 * size_t(col) * g.ldc + rr]
                                       : T(0);
                }
            }
    }

    // operand selection for this lane (see the header comment)
    const int s = lane & 1;                  // real row parity: 0 = re row, 1 = im row
    const int u = (lane >> 4) & 1;           // real k parity:   0 = re k,   1 = im k
    const int kq = lane >> 5;                // which of the 2 complex k of an MFMA step
    const bool take_im_a = (s ^ u) != 0;
    const T sign_a = ((s == 0 && u == 1) ? T(-1) : T(1)) * g.alpha;
    const int a_row = (lane & 15) >> 1;      // complex row within an 8-row block

    const int nchunks = (g.K + BK - 1) / BK;
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) load_chunk((c + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 2) {
            const int k = kk + kq;
            T av[RB], bv[CB];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const ct a = As[buf][k][wr + i * 8 + a_row];
                av[i] = sign_a * (take_im_a ? a.y : a.x);
            }
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const ct b = Bs[buf][wc + j * 16 + b_col][k];
                bv[j] = u ? b.y : b.x;
            }
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < CB; ++j) acc[i][j] = Mfma<T>::op(av[i], bv[j], acc[i][j]);
        }
        if (c + 1 < nchunks) store_chunk(buf ^ 1);
        __syncthreads();
    }

    // epilogue in the real view of the interleaved storage: real row 2i + part
    // is exactly the MFMA output row
    T* Dr = g.D + 2 * (size_t(bz) * g.sD + size_t(bi) * g.sD2);
#pragma unroll
    for (int i = 0; i < RB; ++i) {
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int col = col0 + wc + j * 16 + b_col;
            if (col >= g.N) continue;
            const int rbase = 2 * (row0 + wr + i * 8);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = rbase + Mfma<T>::out_row(lane, v);
                if (rr < M2) Dr[2 * size_t(col) * g.ldd + rr] = acc[i][j][v];
            }
        }
    }
}

template <typename T> struct GemmTile;
template <> struct GemmTile<float> {
    static constexpr int BM = 64, BN = 64, BK = 16;
};
template <> struct GemmTile<double> {
    static constexpr int BM = 32, BN = 64, BK = 16;
};

// Enqueue D = beta C + alpha A B for `batch` (x g.inner) matrices.  M, N, K
// may be zero.  eff_batch (< 0: batch) is the number of outer matrices not
// skipped by g.active, used only for the work accounting of the profiler.
template <typename T>
inline harp_status cgemm(const GemmArgs<T>& g, int batch, hipStream_t stream, int eff_batch = -1) {
    if (g.M <= 0 || g.N <= 0 || batch <= 0 || g.inner <= 0) return HARP_OK;
    if (int64_t(batch) * g.inner > 65535) return HARP_E_ARG;
    constexpr int BM = GemmTile<T>::BM, BN = GemmTile<T>::BN, BK = GemmTile<T>::BK;
    const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    // K == 0 runs the same kernel with an empty contraction: D = beta C
    const double nb = double(eff_batch < 0 ? batch : eff_batch) * g.inner;
    HARP_PROF_LAUNCH(sizeof(T) == 4 ? HARP_K_GEMM32 : HARP_K_GEMM64, stream,
                     8.0 * double(g.M) * double(g.N) * double(g.K) * nb, 0.0,
                     hipLaunchKernelGGL((cgemm_kernel<T, BM, BN, BK>),
                                        dim3(unsigned(tiles), 1u, unsigned(batch * g.inner)), dim3(256), 0, stream,
                                        g));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

}  // namespace harp
