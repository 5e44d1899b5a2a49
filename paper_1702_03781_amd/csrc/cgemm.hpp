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
// Tiling: 256 threads = WM x WN waves over a BM x BN complex workgroup tile;
// K streamed in BK-wide complex chunks through double-buffered LDS (A chunk
// stored [k][row] with its k-rows 16 banks apart, B chunk [col][k] with
// 16-byte aligned columns).  Global loads and the f32 C/D accesses move 16
// bytes per lane (two complex64 or one complex128) when the operands are
// aligned; each lane reads from LDS only the real component it feeds; the
// register fragments of the next MFMA step are read while the current step's
// MFMAs issue.  Each wave owns (BM/WM) x (BN/WN): (BM/WM/8) x (BN/WN/16)
// MFMA blocks.  Small, register-light tiles keep four waves per SIMD, which
// on this hardware beats larger tiles for the rank-64 LU updates.
#pragma once

#include <algorithm>

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
    // A triangular (1: zero above its diagonal, 2: zero below it): a tile row
    // contracts only over the K range where its rows of A can be non-zero
    // (whole zero chunks skipped; the products left out are exact zeros)
    int tri = 0;
    int site = 0;                // call site tag of the kernel timers (harp_prof.h)
    int small_grid = 1024;       // grids of fewer 64 x 64 tiles than this take 32 x 32 tiles
    // T = double only: A held as complex64 (A must be null), each entry
    // widened to FP64 as it is loaded; lda and sA count complex64 elements
    const float* A32 = nullptr;
    // optional [outer batch][N] flags (batch stride s_nz), 0 where that
    // column of B is exactly zero: a tile whose columns are all flagged 0
    // adds an exactly zero product, so it skips the contraction (D = beta C),
    // and an update in place (D == C, beta = 1) ends at once
    const int32_t* b_nz = nullptr;
    int64_t s_nz = 0;
};

template <typename T> struct alignas(16) Vec16 {
    typename Mfma<T>::c_t v[16 / sizeof(typename Mfma<T>::c_t)];
};

template <typename T, int BM, int BN, int BK, int WM, int WN, bool VEC, int OCC = 1, bool PF2 = false,
          bool XCD = false, bool A32 = false>
__global__ void __launch_bounds__(256, OCC) cgemm_kernel(GemmArgs<T> g) {
    static_assert(!A32 || sizeof(T) == 8, "a complex64 A operand is widened for FP64 products only");
    static_assert(!A32 || (BM * BK) % 512 == 0, "complex64 A: whole 16-byte pairs of rows per thread");
    using ct = typename Mfma<T>::c_t;
    using acc_t = typename Mfma<T>::acc_t;
    constexpr int NV = int(16 / sizeof(ct));          // complex per 16-byte access
    constexpr int WTM = BM / WM, WTN = BN / WN;       // wave tile
    constexpr int RB = WTM / 8, CB = WTN / 16;        // MFMA blocks per wave
    constexpr int NA = BM * BK / NV / 256;            // A vectors per thread per chunk
    constexpr int NBv = BN * BK / NV / 256;           // B vectors per thread per chunk
    constexpr int APAD = 8 / (int(sizeof(ct)) / 8);   // k-row stride = 16 banks mod 64
    constexpr int BPAD = NV;                          // keeps B columns 16-byte aligned
    constexpr int KS = BK / 2;                        // MFMA steps per chunk
    static_assert(WM * WN == 4, "four waves");
    static_assert(BM % BK == 0, "triangular contraction ranges start and end on chunk boundaries");
    static_assert(WTM % 8 == 0 && WTN % 16 == 0 && BK % NV == 0 && BK % 2 == 0, "tile shape");
    static_assert(NA >= 1 && NBv >= 1 && NA * NV * 256 == BM * BK && NBv * NV * 256 == BN * BK, "load split");

    // workgroup -> (matrix, tile).  With XCD: consecutive workgroups are
    // dispatched to the eight XCDs in turn, so workgroup L is renumbered so
    // that XCD k takes the k-th eighth of all tiles in matrix order, and within
    // a matrix the tiles run in groups of 8 tile rows (column by column inside
    // a group): the A and B panels a tile reads are then shared by the tiles
    // resident in the same XCD's L2 instead of being fetched by every XCD.
    int zz = blockIdx.z, xx = blockIdx.x;
    const int tiles_m = (g.M + BM - 1) / BM;
    int tm, tn;
    if constexpr (XCD) {
        // 32-bit arithmetic (the host keeps every grid below 2^31 workgroups)
        const unsigned L = blockIdx.x + gridDim.x * blockIdx.z, NT = gridDim.x * gridDim.z;
        if (NT % 8 == 0) {
            const unsigned G = (L % 8) * (NT / 8) + L / 8;
            zz = int(G / gridDim.x);
            xx = int(G % gridDim.x);
        }
        const int tiles_n = (g.N + BN - 1) / BN, GM = 8;
        const int first = (xx / (GM * tiles_n)) * GM, gm = min(GM, tiles_m - first), r = xx % (GM * tiles_n);
        tm = first + r % gm;
        tn = r / gm;
    } else {
        tm = xx % tiles_m;
        tn = xx / tiles_m;
    }
    const int bz = zz / g.inner, bi = zz % g.inner;
    if (g.active && g.active[bz] == 0) return;
    const int row0 = tm * BM, col0 = tn * BN;
    bool zero_b = false;   // every wave reads the same flags: uniform
    if (g.b_nz) {
        const int c = col0 + int(threadIdx.x & 63);
        const bool nz = int(threadIdx.x & 63) < BN && c < g.N && g.b_nz[size_t(bz) * g.s_nz + c] != 0;
        zero_b = __builtin_amdgcn_ballot_w64(nz) == 0;
        if (zero_b && g.beta == T(1) && static_cast<const void*>(g.C) == static_cast<const void*>(g.D) &&
            g.ldc == g.ldd && g.sC == g.sD)
            return;
    }

    const size_t a_off = size_t(bz) * g.sA + size_t(bi) * g.sA2;
    // Whether a tile's operand panels lie wholly inside the matrices, and a
    // chunk's K range inside K, is the same for the whole workgroup: such
    // chunks take unguarded 16-byte loads, the others guarded loads of one
    // complex number each.  (A per-lane choice between the two would run both
    // under lane masks into the same registers, and every load would then
    // wait for the one before it.)
    const bool a_full = VEC && row0 + BM <= g.M;
    const bool b_full = VEC && col0 + BN <= g.N;
    const ct* A = A32 ? nullptr : reinterpret_cast<const ct*>(g.A) + a_off;
    const float2* Aw = A32 ? reinterpret_cast<const float2*>(g.A32) + a_off : nullptr;
    const ct* B = reinterpret_cast<const ct*>(g.B) + size_t(bz) * g.sB + size_t(bi) * g.sB2;

    __shared__ __attribute__((aligned(16))) ct As[2][BK][BM + APAD];
    __shared__ __attribute__((aligned(16))) ct Bs[2][BN][BK + BPAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave % WM) * WTM;
    const int wc = (wave / WM) * WTN;

    // global -> registers: A vector e covers rows a_r[e]..+NV-1 of k-row a_k[e];
    // B vector e covers k b_k[e]..+NV-1 of column b_c[e]
    Vec16<T> ra[NA], rb[NBv];
    auto load_chunk = [&](int k0, Vec16<T> (&ra)[NA], Vec16<T> (&rb)[NBv]) {
        const bool k_full = k0 + BK <= g.K;
        if constexpr (!A32) {
            if (a_full && k_full) {
#pragma unroll
                for (int e = 0; e < NA; ++e) {
                    const int v = tid + 256 * e;
                    const int kk = v / (BM / NV), r = (v % (BM / NV)) * NV;
                    ra[e] = *reinterpret_cast<const Vec16<T>*>(A + size_t(k0 + kk) * g.lda + row0 + r);
                }
            } else {
#pragma unroll
                for (int e = 0; e < NA; ++e) {
                    const int v = tid + 256 * e;
                    const int kk = v / (BM / NV), r = (v % (BM / NV)) * NV;
                    const int gk = k0 + kk, gr = row0 + r;
                    const ct* src = A + size_t(gk) * g.lda + gr;
#pragma unroll
                    for (int q = 0; q < NV; ++q)
                        ra[e].v[q] = (gk < g.K && gr + q < g.M) ? src[q] : ct{T(0), T(0)};
                }
            }
        } else {
            // complex64 A: two consecutive rows per thread; the raw bytes wait
            // in register slot 2 e2 and are widened only when stored (after
            // the current chunk's products), so that the loads stay in flight
            // during them
#pragma unroll
            for (int e2 = 0; e2 < NA / 2; ++e2) {
                const int v = tid + 256 * e2;
                const int kk = v / (BM / 2), r = (v % (BM / 2)) * 2;
                const int gk = k0 + kk, gr = row0 + r;
                const float2* src = Aw + size_t(gk) * g.lda + gr;
                char* slot = reinterpret_cast<char*>(&ra[2 * e2]);
                if (a_full && k_full) {
                    const float4 q = *reinterpret_cast<const float4*>(src);
                    __builtin_memcpy(slot, &q, sizeof(q));
                } else {
                    const float2 w0 = (gk < g.K && gr < g.M) ? src[0] : float2{0.f, 0.f};
                    const float2 w1 = (gk < g.K && gr + 1 < g.M) ? src[1] : float2{0.f, 0.f};
                    __builtin_memcpy(slot, &w0, sizeof(w0));
                    __builtin_memcpy(slot + sizeof(w0), &w1, sizeof(w1));
                }
            }
        }
        if (b_full && k_full) {
#pragma unroll
            for (int e = 0; e < NBv; ++e) {
                const int v = tid + 256 * e;
                const int c = v / (BK / NV), kk = (v % (BK / NV)) * NV;
                rb[e] = *reinterpret_cast<const Vec16<T>*>(B + size_t(col0 + c) * g.ldb + k0 + kk);
            }
        } else {
#pragma unroll
            for (int e = 0; e < NBv; ++e) {
                const int v = tid + 256 * e;
                const int c = v / (BK / NV), kk = (v % (BK / NV)) * NV;
                const int gc = col0 + c, gk = k0 + kk;
                const ct* src = B + size_t(gc) * g.ldb + gk;
#pragma unroll
                for (int q = 0; q < NV; ++q)
                    rb[e].v[q] = (gc < g.N && gk + q < g.K) ? src[q] : ct{T(0), T(0)};
            }
        }
    };
    auto store_chunk = [&](int buf, const Vec16<T> (&ra)[NA], const Vec16<T> (&rb)[NBv]) {
        if constexpr (A32) {
#pragma unroll
            for (int e2 = 0; e2 < NA / 2; ++e2) {
                const int v = tid + 256 * e2;
                const int kk = v / (BM / 2), r = (v % (BM / 2)) * 2;
                float4 q;
                __builtin_memcpy(&q, &ra[2 * e2], sizeof(q));
                As[buf][kk][r] = ct{T(q.x), T(q.y)};
                As[buf][kk][r + 1] = ct{T(q.z), T(q.w)};
            }
        } else {
#pragma unroll
            for (int e = 0; e < NA; ++e) {
                const int v = tid + 256 * e;
                const int kk = v / (BM / NV), r = (v % (BM / NV)) * NV;
                *reinterpret_cast<Vec16<T>*>(&As[buf][kk][r]) = ra[e];
            }
        }
#pragma unroll
        for (int e = 0; e < NBv; ++e) {
            const int v = tid + 256 * e;
            const int c = v / (BK / NV), kk = (v % (BK / NV)) * NV;
            *reinterpret_cast<Vec16<T>*>(&Bs[buf][c][kk]) = rb[e];
        }
    };

    // accumulators: beta * C first (PF2: added after the contraction, so that
    // the C read does not wait in front of it); f32 outputs of a lane are four
    // consecutive real rows (one 16-byte access when aligned and in range)
    const int b_col = lane & 15;
    const int M2 = 2 * g.M;
    acc_t acc[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = acc_t{T(0), T(0), T(0), T(0)};
    auto add_c = [&]() {
        const T* Cr = g.C ? g.C + 2 * (size_t(bz) * g.sC + size_t(bi) * g.sC2) : nullptr;
        const bool use_c = g.beta != T(0) && Cr != nullptr;
        if constexpr (sizeof(T) == 4) {
            // a tile wholly inside M and N (the same for the whole workgroup):
            // every 16-byte C access is issued before the first is used
            if (use_c && a_full && b_full) {
                f32x4 c4[RB][CB];
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < CB; ++j) {
                        const int col = col0 + wc + j * 16 + b_col;
                        const int r4 = 2 * (row0 + wr + i * 8) + 4 * (lane >> 4);
                        c4[i][j] = *reinterpret_cast<const f32x4*>(Cr + 2 * size_t(col) * g.ldc + r4);
                    }
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < CB; ++j) acc[i][j] += c4[i][j] * g.beta;
                return;
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int col = col0 + wc + j * 16 + b_col;
                const int rbase = 2 * (row0 + wr + i * 8);
                if (!use_c || col >= g.N) continue;
                const T* cp = Cr + 2 * size_t(col) * g.ldc;
                if constexpr (sizeof(T) == 4) {
                    const int r4 = rbase + 4 * (lane >> 4);
                    if (VEC && r4 + 4 <= M2) {
                        const f32x4 c4 = *reinterpret_cast<const f32x4*>(cp + r4);
                        acc[i][j] += c4 * g.beta;
                        continue;
                    }
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = rbase + Mfma<T>::out_row(lane, v);
                    if (rr < M2) acc[i][j][v] += g.beta * cp[rr];
                }
            }
    };

    // operand selection for this lane (see the header comment)
    const int s = lane & 1;
    const int u = (lane >> 4) & 1;
    const int kq = lane >> 5;
    const bool take_im_a = (s ^ u) != 0;
    const T sign_a = ((s == 0 && u == 1) ? T(-1) : T(1)) * g.alpha;
    const int a_row = (lane & 15) >> 1;

    // each lane reads only the component it feeds (half the LDS traffic of
    // reading whole complex numbers)
    T fa[2][RB], fb[2][CB];
    const int a_part = take_im_a ? 1 : 0;
    auto frag = [&](int buf, int step, T (&av)[RB], T (&bv)[CB]) {
        const int k = 2 * step + kq;
        const T* ap = reinterpret_cast<const T*>(&As[buf][k][wr + a_row]) + a_part;
#pragma unroll
        for (int i = 0; i < RB; ++i) av[i] = sign_a * ap[2 * 8 * i];
#pragma unroll
        for (int j = 0; j < CB; ++j) bv[j] = reinterpret_cast<const T*>(&Bs[buf][wc + j * 16 + b_col][k])[u];
    };

    auto compute = [&](int buf) {
        frag(buf, 0, fa[0], fb[0]);
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            if (st + 1 < KS) frag(buf, st + 1, fa[(st + 1) & 1], fb[(st + 1) & 1]);
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < CB; ++j) acc[i][j] = Mfma<T>::op(fa[st & 1][i], fb[st & 1][j], acc[i][j]);
        }
    };
    // contraction range of this tile row (row0 and row0 + BM are multiples of BK)
    const int kb = g.tri == 2 ? min(g.K, row0) : 0;
    const int ke = g.tri == 1 ? min(g.K, row0 + BM) : g.K;
    const int nchunks = zero_b ? 0 : (ke - kb + BK - 1) / BK;
    if constexpr (!PF2) {
        // the first chunk's loads go out before the C reads, so that the two
        // are in flight together
        if (nchunks > 0) load_chunk(kb, ra, rb);
        add_c();
        if (nchunks > 0) store_chunk(0, ra, rb);
        __syncthreads();
        for (int c = 0; c < nchunks; ++c) {
            const int buf = c & 1;
            if (c + 1 < nchunks) load_chunk(kb + (c + 1) * BK, ra, rb);
            compute(buf);
            if (c + 1 < nchunks) store_chunk(buf ^ 1, ra, rb);
            __syncthreads();
        }
    } else {
        // two register sets and two LDS buffers: chunk c is loaded into set
        // c & 1 two chunks ahead of its use and stored to buffer c & 1 one
        // chunk ahead (unrolled by two so that every index is a constant)
        Vec16<T> ra1[NA], rb1[NBv];
        if (nchunks > 0) load_chunk(kb, ra, rb);
        if (nchunks > 1) load_chunk(kb + BK, ra1, rb1);
        if (nchunks > 0) store_chunk(0, ra, rb);
        __syncthreads();
        for (int c = 0; c < nchunks; c += 2) {
            if (c + 2 < nchunks) load_chunk(kb + (c + 2) * BK, ra, rb);
            compute(0);
            if (c + 1 < nchunks) store_chunk(1, ra1, rb1);
            __syncthreads();
            if (c + 1 >= nchunks) break;
            if (c + 3 < nchunks) load_chunk(kb + (c + 3) * BK, ra1, rb1);
            compute(1);
            if (c + 2 < nchunks) store_chunk(0, ra, rb);
            __syncthreads();
        }
        add_c();
    }

    T* Dr = g.D + 2 * (size_t(bz) * g.sD + size_t(bi) * g.sD2);
    if constexpr (sizeof(T) == 4) {
        if (a_full && b_full) {   // whole tile: unguarded 16-byte stores
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < CB; ++j) {
                    const int col = col0 + wc + j * 16 + b_col;
                    const int r4 = 2 * (row0 + wr + i * 8) + 4 * (lane >> 4);
                    *reinterpret_cast<f32x4*>(Dr + 2 * size_t(col) * g.ldd + r4) = acc[i][j];
                }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int col = col0 + wc + j * 16 + b_col;
            if (col >= g.N) continue;
            const int rbase = 2 * (row0 + wr + i * 8);
            T* dp = Dr + 2 * size_t(col) * g.ldd;
            if constexpr (sizeof(T) == 4) {
                const int r4 = rbase + 4 * (lane >> 4);
                if (VEC && r4 + 4 <= M2) {
                    *reinterpret_cast<f32x4*>(dp + r4) = acc[i][j];
                    continue;
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = rbase + Mfma<T>::out_row(lane, v);
                if (rr < M2) dp[rr] = acc[i][j][v];
            }
        }
    }
}

// true when every operand row start is 16-byte aligned (pointers, leading
// dimensions and batch strides), so the vector paths of cgemm_kernel apply
template <typename T> inline bool gemm_vec_ok(const GemmArgs<T>& g) {
    constexpr int64_t NV = 16 / (2 * sizeof(T));
    auto al = [](const void* p) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    auto ev = [](int64_t x) { return x % NV == 0; };
    // a complex64 A (FP64 products) is read two rows per 16-byte access
    auto ev2 = [&](int64_t x) { return g.A32 == nullptr || x % 2 == 0; };
    return al(g.A) && al(g.A32) && al(g.B) && al(g.C) && al(g.D) && ev(g.lda) && ev(g.ldb) && ev(g.ldc) &&
           ev(g.ldd) && ev(g.sA) && ev(g.sB) && ev(g.sC) && ev(g.sD) && ev(g.sA2) && ev(g.sB2) && ev(g.sC2) &&
           ev(g.sD2) && ev2(g.lda) && ev2(g.sA) && ev2(g.sA2);
}

// share of the M x K products a triangular A leaves to BM-row tiles
inline double tri_share(int tri, int M, int K, int BM) {
    if (tri == 0 || M <= 0 || K <= 0) return 1.0;
    double done = 0.0;
    for (int r0 = 0; r0 < M; r0 += BM) {
        const int rows = std::min(BM, M - r0);
        const int kb = tri == 2 ? std::min(K, r0) : 0, ke = tri == 1 ? std::min(K, r0 + BM) : K;
        done += double(rows) * (ke - kb);
    }
    return done / (double(M) * K);
}

template <typename T, int BM, int BN, int BK, int WM, int WN, int OCC = 1, bool PF2 = false, bool XCD = false>
inline void launch_cgemm(const GemmArgs<T>& g, int batch, hipStream_t stream, double flops, double bytes) {
    if constexpr (sizeof(T) == 8) {
        if (g.A32) {
            flops *= tri_share(g.tri, g.M, g.K, BM);
            const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
            const dim3 grid(unsigned(tiles), 1u, unsigned(batch * g.inner));
            const int cls = HARP_K_GEMM64 | (g.site << 8);
            if (gemm_vec_ok(g))
                HARP_PROF_EXT_LAUNCH(cls, stream, flops, bytes,
                                     (cgemm_kernel<T, BM, BN, BK, WM, WN, true, OCC, PF2, XCD, true>), grid,
                                     dim3(256), 0, g);
            else
                HARP_PROF_EXT_LAUNCH(cls, stream, flops, bytes,
                                     (cgemm_kernel<T, BM, BN, BK, WM, WN, false, OCC, PF2, XCD, true>), grid,
                                     dim3(256), 0, g);
            return;
        }
    }
    flops *= tri_share(g.tri, g.M, g.K, BM);
    const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    const dim3 grid(unsigned(tiles), 1u, unsigned(batch * g.inner));
    const int cls = (sizeof(T) == 4 ? HARP_K_GEMM32 : HARP_K_GEMM64) | (g.site << 8);
    if (gemm_vec_ok(g))
        HARP_PROF_EXT_LAUNCH(cls, stream, flops, bytes, (cgemm_kernel<T, BM, BN, BK, WM, WN, true, OCC, PF2, XCD>), grid,
                             dim3(256), 0, g);
    else
        HARP_PROF_EXT_LAUNCH(cls, stream, flops, bytes, (cgemm_kernel<T, BM, BN, BK, WM, WN, false, OCC, PF2, XCD>), grid,
                             dim3(256), 0, g);
}

// Enqueue D = beta C + alpha A B for `batch` (x g.inner) matrices.  M, N, K
// may be zero.  eff_batch (< 0: batch) is the number of outer matrices not
// skipped by g.active, used only for the work accounting of the profiler.
// Tile: 64 x 64 (four waves stacked on rows) when that grid has at least
// g.small_grid workgroups (default 1024, four per CU; the LU and solve take it
// from the tuning table); smaller grids (the solve's inverse-block products,
// the LU's thin catch-up, deferred-row and in-block products) take 32 x 32
// tiles for four times the workgroups.  A product in place (D = B) keeps
// 64-row tiles so that one workgroup reads a whole column block of B before
// writing it (callers use it with M <= 64), 32 columns wide for twice the
// workgroups; narrow ones (N <= 32) take the same 64 x 32 tile.
template <typename T>
inline harp_status cgemm(const GemmArgs<T>& g, int batch, hipStream_t stream, int eff_batch = -1) {
    if (g.M <= 0 || g.N <= 0 || batch <= 0 || g.inner <= 0) return HARP_OK;
    if (int64_t(batch) * g.inner > 65535) return HARP_E_ARG;
    // the kernel numbers workgroups in 32 bits (the 32 x 32 tiling has the most)
    if (int64_t((g.M + 31) / 32) * ((g.N + 31) / 32) * batch * g.inner >= (int64_t(1) << 31)) return HARP_E_ARG;
    // K == 0 runs the same kernel with an empty contraction: D = beta C
    const double nb = double(eff_batch < 0 ? batch : eff_batch) * g.inner;
    // algorithmic bytes: A and B read once, C read when beta != 0, D written
    if (g.A32 && (sizeof(T) != 8 || g.A)) return HARP_E_ARG;
    // zero-column flags are per outer matrix
    if (g.b_nz && g.inner != 1) return HARP_E_ARG;
    const bool reads_c = g.beta != T(0) && g.C != nullptr;
    const double a_bytes = g.A32 ? 8.0 : 2.0 * sizeof(T);
    const double bytes = nb * (a_bytes * double(g.M) * g.K +
                               2.0 * sizeof(T) * (double(g.K) * g.N + double(g.M) * g.N * (reads_c ? 2.0 : 1.0)));
    const double flops = 8.0 * double(g.M) * double(g.N) * double(g.K) * nb;
    const int64_t wg64 = int64_t((g.M + 63) / 64) * ((g.N + 63) / 64) * batch * g.inner;
    const bool in_place = static_cast<const void*>(g.D) == static_cast<const void*>(g.B);
    if (!in_place && wg64 < g.small_grid)
        launch_cgemm<T, 32, 32, 16, 4, 1>(g, batch, stream, flops, bytes);
    else if (sizeof(T) == 8 && g.K >= 1024 && g.N > 32)
        // long FP64 contractions (the refinement residual): 8-wide K chunks at
        // two workgroups per CU, each chunk fetched two chunks ahead and C
        // added after the contraction (0.82 of the FP64 peak on the
        // 2048 x 256 x 2048 residual against 0.74 with one chunk ahead)
        launch_cgemm<T, 64, 64, 8, 4, 1, 2, true, true>(g, batch, stream, flops, bytes);
    else if (g.N <= 32 || in_place)
        launch_cgemm<T, 64, 32, 16, 4, 1>(g, batch, stream, flops, bytes);
    else
        launch_cgemm<T, 64, 64, 16, 4, 1, 1, false, true>(g, batch, stream, flops, bytes);
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

}  // namespace harp
