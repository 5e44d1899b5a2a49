// Dense reduced solve: blocked LU with partial pivoting, triangular solves and
// FP64 iterative refinement, batched over independent systems (frequencies,
// layouts).
//
// The reduced MoM system of order n = N_a N_m is solved by Gaussian
// elimination, one right-hand side per antenna port (Section I; the solve is
// the O((N_a N_m)^3) part of Section II-B and the "Solving MoM equations" row
// of Table II).
//
// Factorisation (right-looking, outer block nb, inner panels of W columns):
//   for each outer block [k0, k0+nb):
//     for each inner panel [j0, j0+W):
//       getf2_kernel   : pivot search, swap, scale and rank-1 updates of the
//                        panel held in registers (one workgroup per matrix);
//                        the panel's row exchanges applied to the other
//                        columns of the outer block; unit-lower solve of the
//                        outer block's columns to the right of the panel
//       cgemm          : update of the rest of the outer block (MFMA)
//     (the last panel also writes the inverse of the block's unit-lower
//      diagonal block L11 and the block's row-exchange map to a scratch)
//     laswp_kernel     : the block's row exchanges applied to the trailing
//                        columns (and to earlier columns of the solve group)
//     cgemm            : block row U12 = L11^-1 A12, in place (MFMA)
//     cgemm            : trailing update A22 -= L21 U12 (MFMA, the hot loop)
// Row exchanges of a later outer block are not applied to the multipliers of
// earlier blocks; the forward solve applies the exchanges block by block in
// the same order, which is equivalent (the multipliers of block K are stored
// in the row order current at step K).
#include <float.h>
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "cgemm.hpp"
#include "common.hpp"
#include "prof.hpp"

namespace harp {
namespace {

template <typename T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };

template <typename V> __device__ inline V cm(V a, V b) {
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ inline V cfms(V acc, V a, V b) {   // acc - a * b
    acc.x = fma(-a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(-a.x, b.y, fma(-a.y, b.x, acc.y));
    return acc;
}
template <typename V> __device__ inline V crecip(V a) {
    // 1 / a with scaling (Smith's method) to avoid overflow in |a|^2
    using R = decltype(a.x);
    if (fabs(a.x) >= fabs(a.y)) {
        const R r = a.y / a.x, d = a.x + a.y * r;
        return V{R(1) / d, -r / d};
    }
    const R r = a.x / a.y, d = a.y + a.x * r;
    return V{r / d, R(-1) / d};
}

// ---------------------------------------------------------------------------
// panel factorisation
// ---------------------------------------------------------------------------

struct PanelArgs {
    void* A;
    int64_t lda, sA;
    int n, k0, kend, j0, w;
    int32_t* ipiv;      // [batch][n]
    int32_t* info;      // [batch]
    void* blk;          // last panel of an outer block: per-matrix block scratch, else null
};

// widest outer block the panel kernel serves (its LDS staging is sized for it)
constexpr int NBMAX = 64;

// Per-matrix scratch of one outer block, written by its last panel and read
// by the block-row solve: the inverse of the unit-lower diagonal block
// (NBMAX x NBMAX complex, column-major, identity past the block's width) and
// the block's row-exchange map (cand[2 NBMAX]: rows touched; src[2 NBMAX]:
// where each one's content comes from after all the block's exchanges).
template <typename T> struct BlkScratch {
    static constexpr int64_t linv_bytes = int64_t(NBMAX) * NBMAX * 2 * int64_t(sizeof(T));
    static constexpr int64_t stride = ((linv_bytes + 4 * NBMAX * 4) + 255) / 256 * 256;
};

// Wave-wide argmax of (value, row) with the LAPACK tie rule (larger value,
// then smaller row).  DPP moves inside each 16-lane row (quad swaps, then
// rotations by 4 and 8), then the four row results are read as scalars.
// A NaN value never wins a comparison.
template <int CTRL> __device__ inline int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ inline float dpp_v(float v) { return __int_as_float(dpp_i<CTRL>(__float_as_int(v))); }
template <int CTRL> __device__ inline double dpp_v(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>(int(b)), hi = dpp_i<CTRL>(int(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ inline float readlane_v(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ inline double readlane_v(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b), l), hi = __builtin_amdgcn_readlane(int(b >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <typename T> __device__ inline void take_if_better(T ov, int oi, T& best, int& bidx) {
    // branch-free: the selects stay in VALU without exec-mask changes
    const bool t = (ov > best) | ((ov == best) & (oi < bidx));
    best = t ? ov : best;
    bidx = t ? oi : bidx;
}
template <typename T, int CTRL> __device__ inline void dpp_step(T& best, int& bidx) {
    take_if_better(dpp_v<CTRL>(best), dpp_i<CTRL>(bidx), best, bidx);
}
template <typename T> __device__ inline void row16_argmax(T& best, int& bidx) {
    dpp_step<T, 0xB1>(best, bidx);    // quad_perm [1,0,3,2]
    dpp_step<T, 0x4E>(best, bidx);    // quad_perm [2,3,0,1]
    dpp_step<T, 0x124>(best, bidx);   // row_ror:4
    dpp_step<T, 0x128>(best, bidx);   // row_ror:8
}
// row broadcasts: lane 15 of each row into the next row (rows 1 and 3), then
// lane 31 into rows 2 and 3; lane 63 ends with the wave's result.  Rows left
// out by the row mask compare their value with itself (no change).
template <int CTRL, int ROWS> __device__ inline int dpp_rows_i(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS> __device__ inline float dpp_rows_v(float old, float v) {
    return __int_as_float(dpp_rows_i<CTRL, ROWS>(__float_as_int(old), __float_as_int(v)));
}
template <int CTRL, int ROWS> __device__ inline double dpp_rows_v(double old, double v) {
    const long long o = __double_as_longlong(old), b = __double_as_longlong(v);
    const int lo = dpp_rows_i<CTRL, ROWS>(int(o), int(b)), hi = dpp_rows_i<CTRL, ROWS>(int(o >> 32), int(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <typename T, int CTRL, int ROWS> __device__ inline void dpp_bcast_step(T& best, int& bidx) {
    take_if_better(dpp_rows_v<CTRL, ROWS>(best, best), dpp_rows_i<CTRL, ROWS>(bidx, bidx), best, bidx);
}
template <typename T> __device__ inline void wave_argmax(T& best, int& bidx) {
    row16_argmax(best, bidx);
    dpp_bcast_step<T, 0x142, 0xA>(best, bidx);   // row_bcast:15
    dpp_bcast_step<T, 0x143, 0xC>(best, bidx);   // row_bcast:31
    best = readlane_v(best, 63);
    bidx = __builtin_amdgcn_readlane(bidx, 63);
}

// Reciprocal of a pivot.  Single precision: Smith's scaling with the hardware
// reciprocal (about 1 ulp per step; the refinement absorbs it).  Double
// precision: IEEE divisions.
__device__ inline float2 crecip_pivot(float2 a) {
    if (fabsf(a.x) >= fabsf(a.y)) {
        const float r = a.y * __builtin_amdgcn_rcpf(a.x), d = fmaf(a.y, r, a.x);
        const float id = __builtin_amdgcn_rcpf(d);
        return float2{id, -r * id};
    }
    const float r = a.x * __builtin_amdgcn_rcpf(a.y), d = fmaf(a.x, r, a.y);
    const float id = __builtin_amdgcn_rcpf(d);
    return float2{r * id, -id};
}
__device__ inline double2 crecip_pivot(double2 a) { return crecip(a); }

// Single-precision pivot search on 32-bit keys: the bit pattern of a
// magnitude |re| + |im| (non-negative, so its bits order like its value), or
// -1 for rows outside [j, n) and NaN magnitudes, which then never win.  The
// largest key comes from integer DPP max steps (one VALU operation each), the
// lanes holding it from a ballot; only an exact tie between lanes needs a
// second reduction, a minimum over their row labels, so the smallest row wins
// as in LAPACK.
template <int CTRL, int ROWS> __device__ inline int dpp_any(int v) {
    if constexpr (ROWS == 0xF) {   // every lane written: no old value needed
        return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
    } else {                       // rows left out keep their own value
        return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xF, false);
    }
}
template <int CTRL, int ROWS> __device__ inline void max_step(int& v) { v = max(v, dpp_any<CTRL, ROWS>(v)); }
template <int CTRL, int ROWS> __device__ inline void min_step(int& v) { v = min(v, dpp_any<CTRL, ROWS>(v)); }
// every lane of each 16-lane row ends with the row's maximum / minimum
__device__ inline int row16_max(int v) {
    max_step<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    max_step<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    max_step<0x124, 0xF>(v);   // row_ror:4
    max_step<0x128, 0xF>(v);   // row_ror:8
    return v;
}
__device__ inline int row16_min(int v) {
    min_step<0xB1, 0xF>(v);
    min_step<0x4E, 0xF>(v);
    min_step<0x124, 0xF>(v);
    min_step<0x128, 0xF>(v);
    return v;
}
// the wave's maximum / minimum (uniform)
__device__ inline int wave_max(int v) {
    v = row16_max(v);
    max_step<0x142, 0xA>(v);   // row_bcast:15
    max_step<0x143, 0xC>(v);   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ inline int wave_min(int v) {
    v = row16_min(v);
    min_step<0x142, 0xA>(v);
    min_step<0x143, 0xC>(v);
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ inline uint64_t ballot64(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }

// LDS of the panel kernel (candidates double-buffered by column parity);
// the row buffers come first so their 16-byte vectors stay aligned.  W is
// the width of one register block, WT the panel's whole width (W or 2 W).
template <typename T, int NT, int W, int WT = W> struct alignas(16) PanelShared {
    using V = typename C2<T>::t;
    static constexpr int NW = NT / 64;
    V cand_row[2][NW][W];
    V stage[NBMAX - W][2 * WT];
    V Ls[WT][WT];
    V Ub[W][W];
    T cand_v[2][NW];
    int cand_i[2][NW];
    int piv_s[WT];
    int first_zero;   // 1 + the first column with a zero pivot (0: none)
    int cand_s[2 * WT], src_s[2 * WT];
    int cand2_s[2 * W], src2_s[2 * W];
};

// Columns [c_from, W) of a row held in LDS, read as 16-byte vectors
// (c_from is rounded down to a vector boundary).
template <int W, int C_FROM> __device__ inline void lds_row(const float2* src, float2 (&dst)[W]) {
    const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
    for (int c2 = C_FROM / 2; c2 < W / 2; ++c2) {
        const float4 q = s4[c2];
        dst[2 * c2] = float2{q.x, q.y};
        dst[2 * c2 + 1] = float2{q.z, q.w};
    }
}
template <int W, int C_FROM> __device__ inline void lds_row(const double2* src, double2 (&dst)[W]) {
#pragma unroll
    for (int c = C_FROM; c < W; ++c) dst[c] = src[c];
}

// Column JJ of a register block of the panel (then JJ+1, ...): a compile-time
// recursion, so the register-resident panel is only ever indexed by
// constants.  The block holds the panel's columns [C0, C0 + W).  Row
// exchanges are virtual: lrow[r] is the row that register row r currently
// holds, an exchange of rows j and p swaps two of these labels, and the
// write-back puts every register row at its label.
template <typename T, int NT, int RPT, int W, int WT, int C0, int JJ>
__device__ __forceinline__ void panel_columns(typename C2<T>::t (&a)[RPT][W], int (&lrow)[RPT],
                                              PanelShared<T, NT, W, WT>& sh, const PanelArgs& pa, int b, int tid) {
    if constexpr (JJ < W) {
        using V = typename C2<T>::t;
        constexpr int NW = NT / 64;
        constexpr int par = (C0 + JJ) & 1;
        const int n = pa.n;
        if (C0 + JJ >= pa.w) return;
        const int lane = tid & 63, wave = tid >> 6;
        const int j = pa.j0 + C0 + JJ;
        // wave candidate: the label of its row (-1: the wave has none)
        int bidx = -1;
        T best = T(-1);
        if constexpr (sizeof(T) == 4) {
            // lane candidate: the largest key of its rows, smallest label on a tie
            int key = -1, lab = INT_MAX;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const float m = fabsf(a[r][JJ].x) + fabsf(a[r][JJ].y);
                const int k = (lrow[r] >= j && lrow[r] < n && m == m) ? __float_as_int(m) : -1;
                const bool t = (k > key) | ((k == key) & (lrow[r] < lab));
                key = t ? k : key;
                lab = t ? lrow[r] : lab;
            }
            const int wk = wave_max(key);
            if (wk >= 0) {
                const uint64_t hit = ballot64(key == wk);
                if (__popcll(hit) == 1) {
                    bidx = __builtin_amdgcn_readlane(lab, __ffsll(static_cast<long long>(hit)) - 1);
                } else {
                    bidx = wave_min(key == wk ? lab : INT_MAX);
                }
                best = __int_as_float(wk);
            }
        } else {
            // rows outside [j, n) carry -2 and never win; a NaN never wins a comparison
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const T m = fabs(a[r][JJ].x) + fabs(a[r][JJ].y);
                take_if_better((lrow[r] >= j && lrow[r] < n) ? m : T(-2), lrow[r], best, bidx);
            }
            wave_argmax(best, bidx);
            if (!(best >= T(0))) bidx = -1;   // no qualifying row in this wave
        }
        // the holder of the wave's candidate publishes that row (the columns
        // from JJ on, rounded down to a 16-byte vector, are all that is read)
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (lrow[r] == bidx) {
#pragma unroll
                for (int c = (JJ / 2) * 2; c < W; ++c) sh.cand_row[par][wave][c] = a[r][c];
            }
        }
        if (lane == 0) {
            sh.cand_v[par][wave] = bidx >= 0 ? best : T(-1);
            sh.cand_i[par][wave] = bidx >= 0 ? bidx : INT_MAX;
        }
        __syncthreads();
        // every wave reduces the NW candidates at once (lane q holds wave q's);
        // wb is the wave that published the winner.  No qualifying row at
        // all (a NaN column) is handled like a zero pivot on row j itself.
        int p = j, wb = -1;
        bool zero = true;
        T bv = T(-1);
        int bi = INT_MAX;
        if (lane < NW) {
            bv = sh.cand_v[par][lane];
            bi = sh.cand_i[par][lane];
        }
        if constexpr (sizeof(T) == 4) {
            // candidates' magnitudes are non-negative or -1: their bits order as ints
            const int ck = __float_as_int(bv);
            const int g = __builtin_amdgcn_readlane(row16_max(ck), 0);
            if (g >= 0) {
                const uint64_t hit = ballot64(lane < NW && ck == g);
                if (__popcll(hit) == 1) {
                    wb = __ffsll(static_cast<long long>(hit)) - 1;
                    p = __builtin_amdgcn_readlane(bi, wb);
                } else {
                    p = __builtin_amdgcn_readlane(row16_min(ck == g ? bi : INT_MAX), 0);
                    wb = __ffsll(static_cast<long long>(ballot64(lane < NW && bi == p))) - 1;
                }
                zero = g == 0;
            }
        } else {
            const int mine = bi;
            row16_argmax(bv, bi);
            bv = readlane_v(bv, 0);
            bi = __builtin_amdgcn_readlane(bi, 0);
            const uint64_t hit = __ballot(lane < NW && mine == bi);
            wb = bv >= T(0) ? __ffsll(static_cast<long long>(hit)) - 1 : -1;
            zero = !(bv > T(0));
            p = bv >= T(0) ? bi : j;
        }
        // the pivot and the first zero pivot stay in LDS until the panel ends
        // (no global memory operation inside the column chain)
        if (tid == 0) {
            sh.piv_s[C0 + JJ] = p;
            if (zero && sh.first_zero == 0) sh.first_zero = j + 1;
        }
        // exchange the labels of rows j and p
#pragma unroll
        for (int r = 0; r < RPT; ++r) lrow[r] = lrow[r] == j ? p : (lrow[r] == p ? j : lrow[r]);
        // pivot row (no qualifying row: the zero pivot skips the update, and
        // inv = 0 keeps every multiplier and update zero)
        V prow[W];
        if (wb >= 0) {
            lds_row<W, JJ>(&sh.cand_row[par][wb][0], prow);
        } else {
#pragma unroll
            for (int c = 0; c < W; ++c) prow[c] = V{T(0), T(0)};
        }
        const V inv = !zero ? crecip_pivot(prow[JJ]) : V{T(0), T(0)};
        V l[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            // multipliers below the diagonal; zero above it (no update there)
            const bool below = lrow[r] > j;
            l[r] = below ? cm(a[r][JJ], inv) : V{T(0), T(0)};
            if (below) a[r][JJ] = l[r];
        }
        // rank-1 update (columns past w are zero)
#pragma unroll
        for (int c = JJ + 1; c < W; ++c) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) a[r][c] = cfms(a[r][c], l[r], prow[c]);
        }
        panel_columns<T, NT, RPT, W, WT, C0, JJ + 1>(a, lrow, sh, pa, b, tid);
    }
}

// LDS of the block inverse: M holds L (strictly lower part, M[i][j], i > j)
// and L^-1 transposed (strictly upper part: M[j][i] = L^-1(i, j), i > j) --
// both unit-lower, so one square array holds them -- plus a product buffer.
template <typename T> struct BlkShared {
    using V = typename C2<T>::t;
    V M[NBMAX][NBMAX + 1];
    V tmp[NBMAX / 2][NBMAX / 2 + 1];
    int pv[NBMAX];
};

template <typename V> __device__ inline V cfma(V acc, V a, V b) {   // acc + a * b
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
    return acc;
}

// One level of the blocked inversion: for each of the NBMAX / (2h) diagonal
// blocks of size 2h with inverted h x h diagonal halves A^-1, B^-1 and
// off-diagonal part C of L, the off-diagonal part of the inverse is
// -B^-1 (C A^-1).
template <typename T, int NT, int H>
__device__ inline void linv_level(BlkShared<T>& bs, int tid) {
    using V = typename C2<T>::t;
    constexpr int NBLK = NBMAX / (2 * H);
    static_assert(NBLK * H <= NBMAX / 2, "product buffer");
    // T = C A^-1 : T(i, j) = C(i, j) + sum_{k > j} C(i, k) A^-1(k, j)
    for (int e = tid; e < NBLK * H * H; e += NT) {
        const int blk = e / (H * H), i = (e / H) % H, j = e % H, o = 2 * H * blk;
        V acc = bs.M[o + H + i][o + j];
        for (int k = j + 1; k < H; ++k) acc = cfma(acc, bs.M[o + H + i][o + k], bs.M[o + j][o + k]);
        bs.tmp[blk * H + i][j] = acc;
    }
    __syncthreads();
    // R = -B^-1 T : R(i, j) = -(T(i, j) + sum_{k < i} B^-1(i, k) T(k, j)), stored transposed
    for (int e = tid; e < NBLK * H * H; e += NT) {
        const int blk = e / (H * H), i = (e / H) % H, j = e % H, o = 2 * H * blk;
        V acc = bs.tmp[blk * H + i][j];
        for (int k = 0; k < i; ++k) acc = cfma(acc, bs.M[o + H + k][o + H + i], bs.tmp[blk * H + k][j]);
        bs.M[o + j][o + H + i] = V{-acc.x, -acc.y};
    }
    __syncthreads();
}

// Last panel of an outer block [k0, kend): with the block's unit-lower
// diagonal block now final in A, write its inverse and the block's row
// exchange map to the block scratch.  The inverse is blocked: 16 x 16
// diagonal blocks by substitution (a lane per entry), then two doubling levels
// of products.
template <typename T, int NT>
__device__ void block_finish(const PanelArgs& pa, int b, int tid, BlkShared<T>& bs) {
    using V = typename C2<T>::t;
    static_assert(NT >= 64 && 1024 % NT == 0, "whole 16-lane groups in every pass");
    __syncthreads();   // this workgroup's writes of the panel and its exchanges are visible
    const V* A = reinterpret_cast<const V*>(pa.A) + size_t(b) * pa.sA;
    const int k0 = pa.k0, nbo = pa.kend - pa.k0, n = pa.n;
    char* base = reinterpret_cast<char*>(pa.blk) + size_t(b) * BlkScratch<T>::stride;
    V* G = reinterpret_cast<V*>(base);
    int32_t* map = reinterpret_cast<int32_t*>(base + BlkScratch<T>::linv_bytes);
    for (int e = tid; e < nbo; e += NT) bs.pv[e] = pa.ipiv[size_t(b) * n + k0 + e];
    for (int e = tid; e < NBMAX * NBMAX; e += NT) {
        const int i = e % NBMAX, j = e / NBMAX;
        bs.M[i][j] = (i > j && i < nbo) ? A[size_t(k0 + j) * pa.lda + k0 + i] : V{T(0), T(0)};
    }
    __syncthreads();
    // exchange map: rows touched (the block's rows and its pivot rows) and the
    // source of each after all exchanges, by walking the exchanges backwards
    if (tid < 2 * nbo) {
        const int r = tid < nbo ? k0 + tid : bs.pv[tid - nbo];
        int src = r;
        for (int q = nbo - 1; q >= 0; --q) {
            if (src == k0 + q) src = bs.pv[q];
            else if (src == bs.pv[q]) src = k0 + q;
        }
        map[tid] = r;
        map[2 * NBMAX + tid] = src;
    }
    // 16 x 16 diagonal blocks: column c of block d's inverse by forward
    // substitution with a lane per row i (16-lane groups), x_q taken by a lane
    // shuffle once final; stored transposed in the upper part
    for (int e = tid; e < 4 * 16 * 16; e += NT) {
        const int o = 16 * (e >> 8), c = (e >> 4) & 15, i = e & 15;
        V x = V{i == c ? T(1) : T(0), T(0)};
#pragma unroll
        for (int q = 0; q < 15; ++q) {
            const V xq = V{__shfl(x.x, q, 16), __shfl(x.y, q, 16)};
            if (i > q && q >= c) x = cfms(x, bs.M[o + i][o + q], xq);
        }
        if (i > c) bs.M[o + c][o + i] = x;
    }
    __syncthreads();
    linv_level<T, NT, 16>(bs, tid);
    linv_level<T, NT, 32>(bs, tid);
    for (int e = tid; e < NBMAX * NBMAX; e += NT) {
        const int i = e % NBMAX, j = e / NBMAX;
        G[e] = i > j ? bs.M[j][i] : V{i == j ? T(1) : T(0), T(0)};
    }
}

// One workgroup per matrix factors rows [j0, n) x columns [j0, j0+w) held in
// registers (thread t starts with rows j0 + t + r NT), in H register blocks of
// W columns (w <= H W).  One barrier per column: each wave publishes its best
// candidate together with that row; after the barrier every thread picks the
// winner, the labels of rows j and p are exchanged (no data moves), and all
// threads scale and update.  With two blocks, the second block is loaded
// with the first and, once the first is factored, updated inside the
// workgroup: its rows at the first block's pivot labels are solved with the
// first block's unit-lower top (giving U), every row below subtracts its
// multipliers times U, and the second block is factored like the first.
// One launch then covers 2 W columns, and the outer block's remaining columns
// take one update per 2 W columns.
// true when a panel of RPT rows x W complex values per thread fits the VGPR
// budget of an NT-thread workgroup (512 / (NT / 256) per lane, minus headroom)
template <typename T, int NT, int RPT, int W> constexpr bool panel_fits_r() {
    return RPT * W * 2 * int(sizeof(T) / 4) <= (512 / (NT / 256)) - 64;
}
// widest register block (8, 4, 2 or 1 columns) that RPT rows per thread hold
// within the budget of 1024 threads
template <typename T, int RPT> constexpr int panel_block_w() {
    return panel_fits_r<T, 1024, RPT, 8>() ? 8
           : panel_fits_r<T, 1024, RPT, 4>() ? 4
           : panel_fits_r<T, 1024, RPT, 2>() ? 2 : 1;
}
// A panel of W columns at RPT rows per thread: H = 1 or 2 register blocks of
// WB columns.  When the two blocks do not fit in registers together, the
// first is written back and re-read from memory for the second block's
// update (single precision only).
template <typename T, int W, int RPT> struct PanelSplit {
    static constexpr int WB = W < panel_block_w<T, RPT>() ? W : panel_block_w<T, RPT>();
    static constexpr int H = W / WB;
    static constexpr bool ok =
        WB * H == W && H <= 2 && (H == 1 || panel_fits_r<T, 1024, RPT, W>() || sizeof(T) == 4);
};

template <typename T, int NT, int RPT, int W, int H>
__global__ void __launch_bounds__(NT) getf2_kernel(PanelArgs pa) {
    using V = typename C2<T>::t;
    constexpr int NW = NT / 64;
    constexpr int WT = W * H;
    static_assert(NW <= 16, "candidates are reduced within one 16-lane row");
    static_assert(H == 1 || H == 2, "one or two register blocks");
    static_assert(2 * WT + 2 * W <= NT, "one thread per row of the exchange maps");
    // the two blocks do not fit in registers together: the first block's
    // multipliers are re-read from memory (where this thread wrote them) for
    // the second block's update
    constexpr bool RELOAD = H == 2 && !panel_fits_r<T, NT, RPT, WT>();
    // column k + 1 of the re-read multipliers is loaded while column k is
    // applied, except at 8 rows per thread (the registers are full there;
    // measured the same either way)
    constexpr bool PREFETCH = RPT <= 4;
    const int b = blockIdx.x;
    V* A = reinterpret_cast<V*>(pa.A) + size_t(b) * pa.sA;
    const int64_t lda = pa.lda;
    const int n = pa.n, j0 = pa.j0, w = pa.w;
    const int tid = threadIdx.x;

    __shared__ PanelShared<T, NT, W, WT> sh;
    auto& Ls = sh.Ls;
    auto& piv_s = sh.piv_s;
    auto& cand_s = sh.cand_s;
    auto& src_s = sh.src_s;
    auto& stage = sh.stage;

    constexpr int W2 = H == 2 ? W : 1;   // second block (unused when H == 1)
    V a[RPT][W], a2[RPT][W2];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = j0 + tid + r * NT;
#pragma unroll
        for (int c = 0; c < W; ++c)
            a[r][c] = (row < n && c < w) ? A[size_t(j0 + c) * lda + row] : V{T(0), T(0)};
    }

    int lrow[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) lrow[r] = j0 + tid + r * NT;
    if (tid == 0) sh.first_zero = 0;
    panel_columns<T, NT, RPT, W, WT, 0, 0>(a, lrow, sh, pa, b, tid);
    const int w1 = w < W ? w : W;   // columns of the first block
    const int w2 = w - w1;          // columns of the second (0 with one block)

    // the first block goes back at its labels now (with two blocks the
    // second block's exchanges reach it below, like any other column); its
    // unit-lower top stays in LDS.  A full-width block (the same for the
    // whole workgroup) stores every column of a row in one straight run, so
    // that each store has its own address registers and none waits for the
    // one before it.
    // (the LDS copy first: nothing after the global stores then waits for
    // them to finish)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = lrow[r];
        if (row >= j0 && row < j0 + w1) {
#pragma unroll
            for (int c = 0; c < W; ++c) Ls[row - j0][c] = a[r][c];
        }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = lrow[r];
        if (row < n) {
            if (w1 == W) {
#pragma unroll
                for (int c = 0; c < W; ++c) A[size_t(j0 + c) * lda + row] = a[r][c];
            } else {
#pragma unroll
                for (int c = 0; c < W; ++c)
                    if (c < w1) A[size_t(j0 + c) * lda + row] = a[r][c];
            }
        }
    }
    if constexpr (H == 2) {
        if (w2 > 0) {
            // the second block, loaded once the first is factored (loading it
            // with the first measured no faster and holds 32 more registers
            // through the first block's columns), and its rows at the first
            // block's top labels (the first block's exchanges are label swaps)
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int row = j0 + tid + r * NT;
#pragma unroll
                for (int c = 0; c < W; ++c)
                    a2[r][c] = (row < n && c < w2) ? A[size_t(j0 + W + c) * lda + row] : V{T(0), T(0)};
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int row = lrow[r];
                if (row >= j0 && row < j0 + W) {
#pragma unroll
                    for (int c = 0; c < W; ++c) sh.Ub[row - j0][c] = a2[r][c];
                }
            }
            __syncthreads();
            // U = L11^-1 (those rows): one column per thread
            if (tid < W) {
                V x[W];
#pragma unroll
                for (int i = 0; i < W; ++i) x[i] = sh.Ub[i][tid];
#pragma unroll
                for (int q = 0; q < W; ++q) {
#pragma unroll
                    for (int i = q + 1; i < W; ++i) x[i] = cfms(x[i], Ls[i][q], x[q]);
                }
#pragma unroll
                for (int i = 0; i < W; ++i) sh.Ub[i][tid] = x[i];
            }
            __syncthreads();
            // rows below the first block: a2 -= L U, one row of U at a time
            // (the compiler fence keeps all 64 entries of U from being loaded
            // into registers at once); the top rows of a2 become U.  With
            // RELOAD, column k of L comes from memory.
            if constexpr (RELOAD) {
                V lk[RPT], ln[RPT];
                auto load_l = [&](int k, V (&l)[RPT]) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
                        l[r] = (lrow[r] >= j0 + W && lrow[r] < n) ? A[size_t(j0 + k) * lda + lrow[r]]
                                                                    : V{T(0), T(0)};
                };
                load_l(0, lk);
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    if (PREFETCH && k + 1 < W) load_l(k + 1, ln);
                    V u[W];
#pragma unroll
                    for (int c = 0; c < W; ++c) u[c] = sh.Ub[k][c];
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        if (lrow[r] >= j0 + W) {
#pragma unroll
                            for (int c = 0; c < W; ++c) a2[r][c] = cfms(a2[r][c], lk[r], u[c]);
                        }
                    }
                    if constexpr (PREFETCH) {
#pragma unroll
                        for (int r = 0; r < RPT; ++r) lk[r] = ln[r];
                    } else if (k + 1 < W) {
                        load_l(k + 1, lk);
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                }
            } else {
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    V u[W];
#pragma unroll
                    for (int c = 0; c < W; ++c) u[c] = sh.Ub[k][c];
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        if (lrow[r] >= j0 + W) {
#pragma unroll
                            for (int c = 0; c < W; ++c) a2[r][c] = cfms(a2[r][c], a[r][k], u[c]);
                        }
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                }
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int row = lrow[r];
                if (row >= j0 && row < j0 + W) {
#pragma unroll
                    for (int c = 0; c < W; ++c) a2[r][c] = sh.Ub[row - j0][c];
                }
            }
            panel_columns<T, NT, RPT, W, WT, W2, 0>(a2, lrow, sh, pa, b, tid);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int row = lrow[r];
                if (row >= j0 && row < j0 + w) {
#pragma unroll
                    for (int c = 0; c < W; ++c) Ls[row - j0][W + c] = a2[r][c];
                }
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int row = lrow[r];
                if (row < n) {
                    if (w2 == W) {
#pragma unroll
                        for (int c = 0; c < W; ++c) A[size_t(j0 + W + c) * lda + row] = a2[r][c];
                    } else {
#pragma unroll
                        for (int c = 0; c < W; ++c)
                            if (c < w2) A[size_t(j0 + W + c) * lda + row] = a2[r][c];
                    }
                }
            }
        }
    }
    __syncthreads();

    // the panel's pivots and its first zero pivot (LAPACK's info: the
    // earliest column wins, and panels run in column order)
    if (tid < w) pa.ipiv[size_t(b) * n + j0 + tid] = piv_s[tid];
    if (tid == 0 && sh.first_zero != 0) atomicCAS(pa.info + b, 0, sh.first_zero);
    // rows touched by this panel's exchanges: the w top rows and the w pivot
    // rows; source of each after all exchanges, by walking them backwards.
    // With two blocks, the first block's columns take the second block's
    // exchanges only (map 2: its w2 top rows and w2 pivot rows).
    if (tid < 2 * w) {
        const int r = tid < w ? j0 + tid : piv_s[tid - w];
        int src = r;
        for (int q = w - 1; q >= 0; --q) {
            if (src == j0 + q) src = piv_s[q];
            else if (src == piv_s[q]) src = j0 + q;
        }
        cand_s[tid] = r;
        src_s[tid] = src;
    } else if (tid < 2 * w + 2 * w2) {
        const int t = tid - 2 * w;
        const int r = t < w2 ? j0 + W + t : piv_s[W + t - w2];
        int src = r;
        for (int q = w - 1; q >= W; --q) {
            if (src == j0 + q) src = piv_s[q];
            else if (src == piv_s[q]) src = j0 + q;
        }
        sh.cand2_s[t] = r;
        sh.src2_s[t] = src;
    }
    __syncthreads();

    // other columns of the outer block (then, with two blocks, the first
    // block's columns): gather the exchanged rows through LDS
    const int left = j0 - pa.k0;
    const int right = pa.kend - (j0 + w);
    const int nother = left + right;
    const int n2 = 2 * w, m2 = 2 * w2;
    {
        // every load of a thread before the first of its LDS stores
        constexpr int PER1 = (2 * WT * NBMAX + NT - 1) / NT, PER2 = (2 * W * W + NT - 1) / NT;
        V g1[PER1], g2[PER2];
#pragma unroll
        for (int q = 0; q < PER1; ++q) {
            const int e = tid + NT * q;
            if (e < n2 * nother) {
                const int t = e % n2, oc = e / n2;
                const int col = oc < left ? pa.k0 + oc : j0 + w + (oc - left);
                g1[q] = A[size_t(col) * lda + src_s[t]];
            }
        }
#pragma unroll
        for (int q = 0; q < PER2; ++q) {
            const int e = tid + NT * q;
            if (e < m2 * W) g2[q] = A[size_t(j0 + e / m2) * lda + sh.src2_s[e % m2]];
        }
#pragma unroll
        for (int q = 0; q < PER1; ++q) {
            const int e = tid + NT * q;
            if (e < n2 * nother) stage[e / n2][e % n2] = g1[q];
        }
#pragma unroll
        for (int q = 0; q < PER2; ++q) {
            const int e = tid + NT * q;
            if (e < m2 * W) stage[nother + e / m2][e % m2] = g2[q];
        }
    }
    __syncthreads();
    for (int e = tid; e < n2 * nother; e += NT) {
        const int t = e % n2, oc = e / n2;
        const bool is_right = oc >= left;
        const int col = is_right ? j0 + w + (oc - left) : pa.k0 + oc;
        const int r = cand_s[t];
        // right columns: the top rows are rewritten by the solve below
        if (is_right && r < j0 + w) continue;
        A[size_t(col) * lda + r] = stage[oc][t];
    }
    for (int e = tid; e < m2 * W; e += NT) {
        const int t = e % m2, c = e / m2;
        const int r = sh.cand2_s[t];
        A[size_t(j0 + c) * lda + r] = stage[nother + c][t];
        // the second block's top rows: their first-block multipliers
        if (t < w2) Ls[W + t][c] = stage[nother + c][t];
    }
    __syncthreads();
    // unit-lower solve of the top rows of the right columns: one 16-lane
    // group per column and one lane per row, so the substitution is WT steps
    // of one broadcast (a lane shuffle within the group) and one multiply-add,
    // instead of a chain of WT (WT - 1) / 2 multiply-adds in one lane
    static_assert(WT <= 16, "one lane per top row");
    for (int oc = left + (tid >> 4); oc < nother; oc += NT / 16) {
        const int i = tid & 15;
        const int col = j0 + w + (oc - left);
        const int ic = i < WT ? i : WT - 1;   // rows past the panel: never used
        V x = i < w ? stage[oc][i] : V{T(0), T(0)};
#pragma unroll
        for (int q = 0; q < WT - 1; ++q) {
            const V xq = V{__shfl(x.x, q, 16), __shfl(x.y, q, 16)};
            if (i > q && i < w) x = cfms(x, Ls[ic][q], xq);
        }
        if (i < w) A[size_t(col) * lda + j0 + i] = x;
    }
    if (pa.blk) {
        __shared__ BlkShared<T> bs;
        block_finish<T, NT>(pa, b, tid, bs);
    }
}

// ---------------------------------------------------------------------------
// row exchanges of an outer block applied to other columns, from the exchange
// map its last panel wrote: the 2 nbo rows the exchanges touch are gathered
// (from their sources) and scattered back.  The block row is then solved by
// a matrix-core product with the block's inverse unit-lower diagonal block.
// ---------------------------------------------------------------------------

struct LaswpArgs {
    const void* blk;       // block scratch, BlkScratch<T>::stride bytes per matrix
    int nbo;               // width of the outer block
    void* X;
    int64_t ldx, sX;
    int c_begin, c_end;    // columns [c_begin, c_end) ...
    int l_begin, l_end;    // ... and [l_begin, l_end) take the exchanges
};

// Columns per exchange workgroup: 64 bytes of each column row.  The scattered
// 8- or 16-byte accesses are latency-bound, so many small workgroups (8 KB of
// LDS each) beat few large ones: 64-column tiles took 2.6x as long per step.
template <typename T> struct LaswpCols { static constexpr int CB = 8 * 8 / int(2 * sizeof(T)); };

template <typename T>
__global__ void __launch_bounds__(256) laswp_kernel(LaswpArgs la) {
    using V = typename C2<T>::t;
    constexpr int CB = LaswpCols<T>::CB;
    const int b = blockIdx.y;
    const int32_t* map = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(la.blk) +
                                                          size_t(b) * BlkScratch<T>::stride +
                                                          BlkScratch<T>::linv_bytes);
    V* X = reinterpret_cast<V*>(la.X) + size_t(b) * la.sX;
    const int nbo = la.nbo, tid = threadIdx.x, n2 = 2 * nbo;
    // the first tiles take the columns [l_begin, l_end)
    const int left_tiles = (la.l_end - la.l_begin + CB - 1) / CB;
    const bool left = int(blockIdx.x) < left_tiles;
    const int c0 = left ? la.l_begin + blockIdx.x * CB : la.c_begin + (blockIdx.x - left_tiles) * CB;
    const int ncols = min(CB, (left ? la.l_end : la.c_end) - c0);
    __shared__ V S[CB][2 * NBMAX + 1];
    __shared__ int cand[2 * NBMAX], src[2 * NBMAX];
    if (tid < n2) {
        cand[tid] = map[tid];
        src[tid] = map[2 * NBMAX + tid];
    }
    __syncthreads();
    // every load of a thread is issued before the first of its LDS stores
    constexpr int PER = (2 * NBMAX * CB + 255) / 256;
    V v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        if (e < n2 * ncols) v[q] = X[size_t(c0 + e / n2) * la.ldx + src[e % n2]];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        if (e < n2 * ncols) S[e / n2][e % n2] = v[q];
    }
    __syncthreads();
    const int top_end = cand[0] + nbo;   // cand[0] is the block's first row
    for (int e = tid; e < n2 * ncols; e += 256) {
        const int t = e % n2, c = e / n2;
        const int r = cand[t];
        if (t >= nbo && r < top_end) continue;   // written by its top-row entry
        X[size_t(c0 + c) * la.ldx + r] = S[c][t];
    }
}

// ---------------------------------------------------------------------------
// Update of the rest of an outer block after one of its panels:
//   A[j0+w:n, j0+w:c_end) -= A[j0+w:n, j0:j0+w) A[j0:j0+w, j0+w:c_end),  w <= W.
// A contraction of at most W is a few flops per byte, so this is an HBM
// stream, not a matrix-core product: one row per thread (the column-major
// loads and stores of a wave are 64 consecutive rows), CN columns per
// workgroup with their W x CN block of U broadcast from LDS, and every load of
// a thread issued before its first store.  The regions read (the panel's
// columns, the strip's rows) and written are disjoint.
// ---------------------------------------------------------------------------

struct RankArgs {
    void* A;
    int64_t lda, sA;
    int n, j0, w, c_end;
};

template <typename T, int W, int CN>
__global__ void __launch_bounds__(256) rank_update_kernel(RankArgs ra) {
    using V = typename C2<T>::t;
    const int b = blockIdx.z;
    V* A = reinterpret_cast<V*>(ra.A) + size_t(b) * ra.sA;
    const int64_t lda = ra.lda;
    const int j0 = ra.j0, w = ra.w, r0 = j0 + w;
    const int cb = r0 + int(blockIdx.y) * CN;
    const int ncol = min(CN, ra.c_end - cb);
    const int i = r0 + int(blockIdx.x) * 256 + int(threadIdx.x);
    __shared__ V u[W][CN];
    if (threadIdx.x < W * CN) {
        const int k = threadIdx.x / CN, c = threadIdx.x % CN;
        u[k][c] = (k < w && c < ncol) ? A[size_t(cb + c) * lda + j0 + k] : V{T(0), T(0)};
    }
    V l[W], cv[CN];
    const bool row = i < ra.n;
#pragma unroll
    for (int k = 0; k < W; ++k) l[k] = (row && k < w) ? A[size_t(j0 + k) * lda + i] : V{T(0), T(0)};
#pragma unroll
    for (int c = 0; c < CN; ++c) cv[c] = (row && c < ncol) ? A[size_t(cb + c) * lda + i] : V{T(0), T(0)};
    __syncthreads();
    if (!row) return;
#pragma unroll
    for (int c = 0; c < CN; ++c) {
        if (c >= ncol) break;
        V acc = cv[c];
#pragma unroll
        for (int k = 0; k < W; ++k) acc = cfms(acc, l[k], u[k][c]);
        A[size_t(cb + c) * lda + i] = acc;
    }
}

template <typename T>
harp_status launch_rank_update(void* A, int64_t lda, int64_t sA, int n, int j0, int w, int c_end, int batch,
                               hipStream_t st) {
    constexpr int CN = 4;
    const int M = n - j0 - w, N = c_end - j0 - w;
    if (w < 1 || w > 16 || M <= 0 || N <= 0) return HARP_E_ARG;
    const dim3 grid(unsigned((M + 255) / 256), unsigned((N + CN - 1) / CN), unsigned(batch));
    const double bytes = double(batch) * double(2 * sizeof(T)) * (2.0 * M * N + double(M) * w + double(w) * N);
    const double flops = 8.0 * double(batch) * M * N * w;
    RankArgs ra{A, lda, sA, n, j0, w, c_end};
    if (w <= 8) {
        HARP_PROF_EXT_LAUNCH(HARP_K_RANK, st, flops, bytes, (rank_update_kernel<T, 8, CN>), grid, dim3(256), 0, ra);
    } else {
        HARP_PROF_EXT_LAUNCH(HARP_K_RANK, st, flops, bytes, (rank_update_kernel<T, 16, CN>), grid, dim3(256), 0, ra);
    }
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

// ---------------------------------------------------------------------------
// inverses of the diagonal blocks (solve groups of SB rows)
//
// After the factorisation the unit-lower and upper SB x SB diagonal blocks of
// every group are copied (identity beyond n) and inverted in place by
// recursive doubling: 16 x 16 blocks by substitution, then for s = 32..SB
//   L: [[A, 0], [C, D]]^-1 = [[A^-1, 0], [-D^-1 C A^-1, D^-1]]
//   U: [[A, B], [0, D]]^-1 = [[A^-1, -A^-1 B D^-1], [0, D^-1]]
// with the two products on the matrix cores.  The solves then apply each
// group with matrix-core products instead of substitution.
// ---------------------------------------------------------------------------

constexpr int kSB = 256;         // rows of a solve group
constexpr int kInv0 = 16;        // base block inverted by substitution

// per (matrix, group) record: [Linv SBxSB | Uinv SBxSB | temp SB*SB/4]
constexpr int64_t kRec = 2 * int64_t(kSB) * kSB + int64_t(kSB) * kSB / 4;

template <typename T>
__global__ void __launch_bounds__(256) extract_diag_kernel(const T* __restrict__ LUr, int64_t lda, int64_t sA,
                                                           int n, int G, T* __restrict__ aux) {
    using V = typename C2<T>::t;
    // blockIdx.x = group * kXCols + column chunk: kSB / kXCols columns each
    constexpr int kXCols = 16;
    const int g = blockIdx.x / kXCols, j0 = (blockIdx.x % kXCols) * (kSB / kXCols), b = blockIdx.y;
    const V* LU = reinterpret_cast<const V*>(LUr) + size_t(b) * sA;
    V* rec = reinterpret_cast<V*>(aux) + (size_t(b) * G + g) * kRec;
    V* Lb = rec;
    V* Ub = rec + int64_t(kSB) * kSB;
    for (int e = j0 * kSB + threadIdx.x; e < (j0 + kSB / kXCols) * kSB; e += 256) {
        const int i = e % kSB, j = e / kSB;
        const int gi = g * kSB + i, gj = g * kSB + j;
        const bool in = gi < n && gj < n;
        const V v = in ? LU[size_t(gj) * lda + gi] : V{T(0), T(0)};
        const V one{T(1), T(0)}, zero{T(0), T(0)};
        Lb[e] = (i == j) ? one : ((i > j && in) ? v : zero);
        Ub[e] = (i <= j && in) ? v : ((i == j) ? one : zero);
    }
}

// one workgroup inverts one 16 x 16 diagonal block of Linv (z = 0) or Uinv (z = 1)
template <typename T>
__global__ void __launch_bounds__(64) tri_inv16_kernel(T* __restrict__ aux, int G) {
    using V = typename C2<T>::t;
    const int blk = blockIdx.x % (kSB / kInv0), rg = blockIdx.x / (kSB / kInv0);   // rg = b * G + g
    const bool upper = blockIdx.z == 1;
    V* M = reinterpret_cast<V*>(aux) + size_t(rg) * kRec + (upper ? int64_t(kSB) * kSB : 0);
    V* D = M + size_t(blk) * kInv0 * (kSB + 1);   // top-left of the 16 x 16 block, ld kSB
    __shared__ V a[kInv0][kInv0 + 1];
    const int t = threadIdx.x;
    for (int e = t; e < kInv0 * kInv0; e += 64) a[e % kInv0][e / kInv0] = D[size_t(e / kInv0) * kSB + e % kInv0];
    __syncthreads();
    if (t >= kInv0) return;
    const int j = t;   // this thread's column of the inverse
    V x[kInv0];
#pragma unroll
    for (int i = 0; i < kInv0; ++i) x[i] = V{T(0), T(0)};
    if (!upper) {
        x[j] = V{T(1), T(0)};
#pragma unroll
        for (int i = 1; i < kInv0; ++i) {
            V acc = x[i];
#pragma unroll
            for (int q = 0; q < i; ++q) acc = cfms(acc, a[i][q], x[q]);
            x[i] = i > j ? acc : x[i];
        }
    } else {
#pragma unroll
        for (int i = kInv0 - 1; i >= 0; --i) {
            V acc = (i == j) ? V{T(1), T(0)} : V{T(0), T(0)};
#pragma unroll
            for (int q = i + 1; q < kInv0; ++q) acc = cfms(acc, a[i][q], x[q]);
            x[i] = i <= j ? cm(acc, crecip(a[i][i])) : V{T(0), T(0)};
        }
    }
#pragma unroll
    for (int i = 0; i < kInv0; ++i) D[size_t(j) * kSB + i] = x[i];
}

// composite row permutation of each solve group: cand[t] = row t of the
// group (t < sb) or its t-sb-th pivot row; src[t] = the row whose content ends
// at cand[t] after the group's exchanges (walking them backwards)
__global__ void __launch_bounds__(256) group_perm_kernel(const int32_t* __restrict__ ipiv, int n, int G,
                                                         int32_t* __restrict__ perm) {
    const int g = blockIdx.x, b = blockIdx.y;
    const int g0 = g * kSB, sb = min(kSB, n - g0);
    const int32_t* pv = ipiv + size_t(b) * n + g0;
    int32_t* cand = perm + (size_t(b) * G + g) * 4 * kSB;
    int32_t* src = cand + 2 * kSB;
    for (int e = threadIdx.x; e < 2 * sb; e += 256) {
        const int r = e < sb ? g0 + e : pv[e - sb];
        int sr = r;
        for (int q = sb - 1; q >= 0; --q) {
            if (sr == g0 + q) sr = pv[q];
            else if (sr == pv[q]) sr = g0 + q;
        }
        cand[e] = r;
        src[e] = sr;
    }
}

// rows [g0, g0 + sb) of X after the group's row exchanges go to Tm (ld SB);
// rows the exchanges push below the group are written back into X; with
// colnz, colnz[b * nrhs + c] records whether column c of Tm holds a non-zero
// (a NaN counts as one)
// right-hand sides per gather workgroup: many small workgroups (the gathered
// rows are latency-bound scattered reads; 16 per workgroup took 2x as long)
constexpr int kGatherCols = 2;
template <typename T>
__global__ void __launch_bounds__(256) group_gather_kernel(const int32_t* __restrict__ perm, int G, int g, int sb,
                                                           T* __restrict__ Xr, int64_t ldx, int64_t sX, int nrhs,
                                                           T* __restrict__ Tr, int64_t sT,
                                                           const int32_t* __restrict__ active,
                                                           int32_t* __restrict__ colnz) {
    using V = typename C2<T>::t;
    constexpr int CG = kGatherCols;
    const int b = blockIdx.y;
    if (active && active[b] == 0) return;
    V* X = reinterpret_cast<V*>(Xr) + size_t(b) * sX;
    V* Tm = reinterpret_cast<V*>(Tr) + size_t(b) * sT;
    const int32_t* cand = perm + (size_t(b) * G + g) * 4 * kSB;
    const int32_t* src = cand + 2 * kSB;
    const int g0 = g * kSB;
    const int c0 = blockIdx.x * CG, ncols = min(CG, nrhs - c0);
    const int tid = threadIdx.x;
    __shared__ V S[CG][2 * kSB + 1];
    const int n2 = 2 * sb;
    // all source rows of a thread, then all its loads, then its LDS stores
    constexpr int PER = (2 * kSB * CG + 255) / 256;
    int sr[PER];
    V v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        sr[q] = e < n2 * ncols ? src[e % n2] : 0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        if (e < n2 * ncols) v[q] = X[size_t(c0 + e / n2) * ldx + sr[q]];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        if (e < n2 * ncols) S[e / n2][e % n2] = v[q];
    }
    __syncthreads();
    if (colnz) {
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            bool nz = false;
            if (c < ncols)
                for (int t = tid; t < sb; t += 256) nz |= S[c][t].x != T(0) || S[c][t].y != T(0);
            const int any = __syncthreads_or(nz);
            if (tid == 0 && c < ncols) colnz[size_t(b) * nrhs + c0 + c] = any;
        }
    }
    for (int e = tid; e < n2 * ncols; e += 256) {
        const int t = e % n2, c = e / n2;
        if (t < sb) {
            Tm[size_t(c0 + c) * kSB + t] = S[c][t];
        } else {
            const int r = cand[t];
            if (r >= g0 + sb) X[size_t(c0 + c) * ldx + r] = S[c][t];
        }
    }
}

// ---------------------------------------------------------------------------
// small helpers: zero info, conversions, Frobenius norms, axpy
// ---------------------------------------------------------------------------

__global__ void zero_i32(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <typename Ti, typename To>
__global__ void __launch_bounds__(256) convert_kernel(const Ti* __restrict__ src, int64_t lds, int64_t ss,
                                                      To* __restrict__ dst, int64_t ldd, int64_t sd, int rows,
                                                      int cols, const int32_t* active) {
    const int b = blockIdx.z;
    if (active && active[b] == 0) return;
    src += size_t(b) * ss;
    dst += size_t(b) * sd;
    // work units of 256 rows of one column (the unit index is uniform, so
    // there is no per-element division)
    const int chunks = (rows + 255) / 256, units = chunks * cols;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int c = u / chunks, r = (u % chunks) * 256 + int(threadIdx.x);
        if (r >= rows) continue;
        const Ti v = src[int64_t(c) * lds + r];
        To o;
        o.x = decltype(o.x)(v.x);
        o.y = decltype(o.y)(v.y);
        dst[int64_t(c) * ldd + r] = o;
    }
}

// X += D (complex128 += complex64 or complex128)
template <typename Vd>
__global__ void __launch_bounds__(256) axpy_kernel(double2* __restrict__ X, int64_t ldx, int64_t sx,
                                                   const Vd* __restrict__ D, int64_t ldd, int64_t sd, int rows,
                                                   int cols, const int32_t* active) {
    const int b = blockIdx.z;
    if (active && active[b] == 0) return;
    X += size_t(b) * sx;
    D += size_t(b) * sd;
    const int chunks = (rows + 255) / 256, units = chunks * cols;   // as in convert_kernel
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int c = u / chunks, r = (u % chunks) * 256 + int(threadIdx.x);
        if (r >= rows) continue;
        const Vd d = D[int64_t(c) * ldd + r];
        double2 x = X[int64_t(c) * ldx + r];
        x.x += double(d.x);
        x.y += double(d.y);
        X[int64_t(c) * ldx + r] = x;
    }
}

// sum of |v|^2 over column-major complex128 matrices: per-block partials.
// blockIdx.y selects the matrix (0: M0, 1: M1), so the residual and the
// solution of a refinement sweep take one launch; matrices whose `active`
// flag is 0 are skipped.
constexpr int kNormBlocks = 1024;
constexpr int kNormSlots = 3;   // partials per matrix: residual, solution, correction
// blocks per matrix: about 16 units (256-row column chunks) per block, at most
// kNormBlocks, so that one large matrix still spreads over the whole chip
inline int norm_blocks(int rows, int cols) {
    const int64_t units = int64_t((rows + 255) / 256) * cols;
    return int(std::max<int64_t>(1, std::min<int64_t>(kNormBlocks, (units + 15) / 16)));
}
__global__ void __launch_bounds__(256) sumsq_partial_kernel(const double2* __restrict__ M0, int64_t ld0, int64_t s0,
                                                            const double2* __restrict__ M1, int64_t ld1, int64_t s1,
                                                            int rows, int cols, double* __restrict__ part,
                                                            const int32_t* __restrict__ active) {
    const int b = blockIdx.z, which = blockIdx.y;
    if (active && active[b] == 0) return;
    const double2* Ma = which ? nullptr : M0 + size_t(b) * s0;
    const double2* Mb = which ? M1 + size_t(b) * s1 : nullptr;
    const int64_t ld = which ? ld1 : ld0;
    // four independent accumulators (four loads in flight per thread), added
    // in a fixed order at the end
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int chunks = (rows + 255) / 256, units = chunks * cols;   // as in convert_kernel
    const int G = int(gridDim.x);
    for (int u0 = blockIdx.x; u0 < units; u0 += 4 * G) {
        double2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int u = u0 + q * G;
            const int c = u / chunks, r = (u % chunks) * 256 + int(threadIdx.x);
            v[q] = double2{0.0, 0.0};
            if (u < units && r < rows) {
                v[q] = which ? Mb[int64_t(c) * ld + r] : Ma[int64_t(c) * ld + r];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = fma(v[q].x, v[q].x, fma(v[q].y, v[q].y, acc[q]));
    }
    double a = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(size_t(b) * kNormSlots + which) * kNormBlocks + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
// Squares of a complex64 matrix (the residual's matrix with the complex64
// fill, or a complex64 correction): two rows per 16-byte access when every
// column start is aligned and the order even (vec2, the same for the whole
// launch), the raw values kept until all four loads of a pass are issued;
// partials as above, into `slot`; matrices whose `active` flag is 0 skipped.
__global__ void __launch_bounds__(256) sumsq_partial_c64_kernel(const float2* __restrict__ M, int64_t ld, int64_t s,
                                                                int rows, int cols, bool vec2,
                                                                double* __restrict__ part, int slot,
                                                                const int32_t* __restrict__ active) {
    const int b = blockIdx.z;
    if (active && active[b] == 0) return;
    const float2* Mb = M + size_t(b) * s;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int pairs = (rows + 1) / 2;
    const int chunks = (pairs + 255) / 256, units = chunks * cols;
    const int G = int(gridDim.x);
    for (int u0 = blockIdx.x; u0 < units; u0 += 4 * G) {
        float4 raw[4];
        if (vec2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int u = u0 + q * G;
                const int c = u / chunks, r = 2 * ((u % chunks) * 256 + int(threadIdx.x));
                raw[q] = (u < units && r < rows) ? *reinterpret_cast<const float4*>(Mb + int64_t(c) * ld + r)
                                                 : float4{0.f, 0.f, 0.f, 0.f};
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int u = u0 + q * G;
                const int c = u / chunks, r = 2 * ((u % chunks) * 256 + int(threadIdx.x));
                const float2* src = Mb + int64_t(c) * ld + r;
                const float2 lo = (u < units && r < rows) ? src[0] : float2{0.f, 0.f};
                const float2 hi = (u < units && r + 1 < rows) ? src[1] : float2{0.f, 0.f};
                raw[q] = float4{lo.x, lo.y, hi.x, hi.y};
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double x0 = raw[q].x, y0 = raw[q].y, x1 = raw[q].z, y1 = raw[q].w;
            acc[q] = fma(x0, x0, fma(y0, y0, fma(x1, x1, fma(y1, y1, acc[q]))));
        }
    }
    double a = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(size_t(b) * kNormSlots + slot) * kNormBlocks + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Sum of the nblk partials p[0..nblk) by one 256-thread workgroup in a fixed
// order (strided per thread, then a fixed tree); every thread gets the sum.
__device__ double block_sum_partials(const double* __restrict__ p, int nblk, double* red) {
    double a = 0.0;
    for (int i = int(threadIdx.x); i < nblk; i += 256) a += p[i];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}
// partials of matrix 0 -> Frobenius norm; one workgroup per matrix
__global__ void __launch_bounds__(256) sumsq_final_kernel(const double* __restrict__ part, double* __restrict__ out,
                                                          int nblk) {
    const int b = blockIdx.x;
    __shared__ double red[4];
    const double sq = block_sum_partials(part + size_t(b) * kNormSlots * kNormBlocks, nblk, red);
    if (threadIdx.x == 0) out[b] = sqrt(sq);
}

// R -= sum of the S complex64 slices P[s] (each n x nrhs, ld n, slice stride
// sp), added in FP64 in slice order (the same order for every element and
// every run); systems whose `active` flag is 0 skipped.
__global__ void __launch_bounds__(256) residual_update_kernel(double2* __restrict__ R, int64_t ldr, int64_t sr,
                                                              const float2* __restrict__ P, int64_t sp,
                                                              int64_t sbp, int S, int rows, int cols,
                                                              const int32_t* __restrict__ active) {
    const int b = blockIdx.z;
    if (active && active[b] == 0) return;
    double2* Rb = R + size_t(b) * sr;
    const float2* Pb = P + size_t(b) * sbp;
    const int64_t total = int64_t(rows) * cols;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
        const int64_t c = e / rows, r = e % rows;
        double sx = 0.0, sy = 0.0;
        for (int q = 0; q < S; ++q) {
            const float2 v = Pb[q * sp + c * rows + r];
            sx += double(v.x);
            sy += double(v.y);
        }
        double2& o = Rb[c * ldr + r];
        o.x -= sx;
        o.y -= sy;
    }
}

// Refinement control on the device.  Every system starts active with a
// zero report; after each residual, the check below turns the norms into the
// relative residual ||R||_F / (||Z||_F ||X||_F) and decides: converged
// (inactive), out of sweeps (inactive), or one more correction (iteration
// count + 1).  Kernels of the sweep skip inactive systems.
__global__ void refine_init_kernel(int32_t* __restrict__ active, harp_refine_report* __restrict__ rep,
                                   double* __restrict__ bnd, int batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    active[b] = 1;
    bnd[b] = 0.0;
    rep[b].iters = 0;
    rep[b].converged = 0;
    rep[b].resid_rel = 0.0;
}
// With dnblk > 0 the residual was updated with complex64 products (R = R_prev
// - Z D): its error bound, bc ||Z||_F ||D||_F + bx ||Z||_F ||X||_F + babs, is
// added to the system's running bound bnd[b] (a full FP64 residual resets it),
// and the system converges only when the residual norm plus that bound meets
// the tolerance.
__global__ void __launch_bounds__(256) refine_check_kernel(const double* __restrict__ part, int nblk, int dnblk,
                                                           const double* __restrict__ znorm, double tol, int max_iter,
                                                           double bc, double babs, double bx,
                                                           double* __restrict__ bnd,
                                                           int32_t* __restrict__ active,
                                                           harp_refine_report* __restrict__ rep) {
    const int b = blockIdx.x;
    if (active[b] == 0) return;   // uniform over the workgroup
    __shared__ double red[4];
    const double sr = block_sum_partials(part + size_t(b) * kNormSlots * kNormBlocks, nblk, red);
    const double sx = block_sum_partials(part + (size_t(b) * kNormSlots + 1) * kNormBlocks, nblk, red);
    const double sd = dnblk > 0 ? block_sum_partials(part + (size_t(b) * kNormSlots + 2) * kNormBlocks, dnblk, red)
                                : 0.0;
    if (threadIdx.x != 0) return;
    bnd[b] = dnblk > 0 ? bnd[b] + bc * znorm[b] * sqrt(sd) + bx * znorm[b] * sqrt(sx) + babs : 0.0;
    const double rn = sqrt(sr), denom = znorm[b] * sqrt(sx);
    const double rel = denom > 0.0 ? rn / denom : (rn == 0.0 ? 0.0 : INFINITY);
    const double relb = denom > 0.0 ? (rn + bnd[b]) / denom : (rn == 0.0 && bnd[b] == 0.0 ? 0.0 : INFINITY);
    rep[b].resid_rel = rel;
    if (relb <= tol) {
        rep[b].converged = 1;
        active[b] = 0;
    } else if (rep[b].iters >= max_iter) {
        active[b] = 0;
    } else {
        rep[b].iters += 1;   // a correction follows
    }
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------

template <typename T> struct LuCfg {
    static constexpr int NB = 64;   // outer block: panels, row exchanges and block-row solve
    static constexpr int NS = 4;    // outer blocks per trailing update (its contraction is NS * NB)
};

// Panel width: the register-resident panel holds RPT x WB complex values per
// thread in each of its one or two register blocks with 1024 threads (64
// VGPRs of budget per lane for a block).  Single precision: 16 columns (two
// blocks of 8) up to 4096 rows, 8 columns (two blocks of 4) up to 8192 rows;
// above 2048 rows the first block is re-read from memory for the second's
// update.  These are the defaults of the tuning table (harp_set_tuning),
// which can choose another feasible width and the GEMM tile switch per order.
template <typename T> inline int default_panel_width(int n) {
    if (sizeof(T) == 4) return n <= 4096 ? 16 : 8;
    return n <= 2048 ? 8 : (n <= 4096 ? 4 : 2);
}


// true when a panel of width W has a launch configuration for every height up
// to n rows (the selection of launch_getf2_w)
template <typename T, int W> constexpr bool panel_feasible_w(int n) {
    if (n <= 1024 * 2) return PanelSplit<T, W, 2>::ok;
    if (n <= 1024 * 4) return PanelSplit<T, W, 2>::ok && PanelSplit<T, W, 4>::ok;
    if (n <= 1024 * 8) return PanelSplit<T, W, 2>::ok && PanelSplit<T, W, 4>::ok && PanelSplit<T, W, 8>::ok;
    return false;
}
template <typename T> bool panel_feasible(int W, int n) {
    switch (W) {
        case 16: return sizeof(T) == 4 && panel_feasible_w<T, 16>(n);
        case 8: return panel_feasible_w<T, 8>(n);
        case 4: return panel_feasible_w<T, 4>(n);
        case 2: return panel_feasible_w<T, 2>(n);
    }
    return false;
}

// Process-wide tuning table: entries in ascending max_order; an order above
// the last entry (or an empty table) takes the defaults.
constexpr int kMaxTuning = 64;
std::mutex g_tuning_mutex;
harp_tuning_entry g_tuning[kMaxTuning];
int g_n_tuning = 0;

struct Tune {
    int panel_width, small_grid;
};
template <typename T> Tune tuning_for(int n) {
    std::lock_guard<std::mutex> lock(g_tuning_mutex);
    for (int i = 0; i < g_n_tuning; ++i)
        if (n <= g_tuning[i].max_order)
            return Tune{sizeof(T) == 4 ? g_tuning[i].panel_width_c64 : g_tuning[i].panel_width_c128,
                        g_tuning[i].small_grid_wgs};
    return Tune{default_panel_width<T>(n), 1024};
}

// H register blocks of W columns
template <typename T, int NT, int RPT, int W, int H>
harp_status launch_getf2_cfg(const PanelArgs& pa, int batch, hipStream_t st) {
    if constexpr (panel_fits_r<T, NT, RPT, W>() && (H == 1 || panel_fits_r<T, NT, RPT, W * H>() || sizeof(T) == 4)) {
        // algorithmic work: the panel's own elimination (rank-1 updates of
        // m rows x w columns) and the unit-lower solve of the w top rows of
        // the outer block's columns to its right
        const double m = double(pa.n - pa.j0), w = double(pa.w), right = double(pa.kend - pa.j0 - pa.w);
        double fl = 0.0;
        for (int c = 0; c < pa.w; ++c) fl += 8.0 * (m - c - 1.0) * (w - c - 1.0);
        fl = double(batch) * (fl + 4.0 * w * (w - 1.0) * right);
        HARP_PROF_EXT_LAUNCH(HARP_K_GETF2, st, fl, 0.0, (getf2_kernel<T, NT, RPT, W, H>), dim3(batch), dim3(NT),
                             0, pa);
        HARP_LAUNCH_CHECK();
        return HARP_OK;
    }
    return HARP_E_ARG;
}

// Two rows per thread while the panel is at most 2048 rows high (the
// workgroup shrinks with the panel: fewer waves share the per-column
// reductions), then 4 or 8 rows per thread with 1024 threads; each height
// range takes its own split of the W columns into register blocks.
template <typename T, int W>
harp_status launch_getf2_w(const PanelArgs& pa, int batch, hipStream_t st) {
    const int m = pa.n - pa.j0;
    if (pa.w > W) return HARP_E_ARG;
    using S2 = PanelSplit<T, W, 2>;
    using S4 = PanelSplit<T, W, 4>;
    using S8 = PanelSplit<T, W, 8>;
    if (m <= 1024 * 2) {
        if constexpr (S2::ok) {
            if (m <= 256 * 2) return launch_getf2_cfg<T, 256, 2, S2::WB, S2::H>(pa, batch, st);
            if (m <= 512 * 2) return launch_getf2_cfg<T, 512, 2, S2::WB, S2::H>(pa, batch, st);
            return launch_getf2_cfg<T, 1024, 2, S2::WB, S2::H>(pa, batch, st);
        }
        return HARP_E_ARG;
    }
    if (m <= 1024 * 4) {
        if constexpr (S4::ok) return launch_getf2_cfg<T, 1024, 4, S4::WB, S4::H>(pa, batch, st);
        return HARP_E_ARG;
    }
    if (m <= 1024 * 8) {
        if constexpr (S8::ok) return launch_getf2_cfg<T, 1024, 8, S8::WB, S8::H>(pa, batch, st);
        return HARP_E_ARG;
    }
    return HARP_E_ARG;
}

template <typename T>
harp_status launch_getf2(const PanelArgs& pa, int W, int batch, hipStream_t st) {
    if (pa.w > W) return HARP_E_ARG;
    switch (W) {
        case 16:
            if constexpr (sizeof(T) == 4) return launch_getf2_w<T, 16>(pa, batch, st);
            return HARP_E_ARG;
        case 8: return launch_getf2_w<T, 8>(pa, batch, st);
        case 4: return launch_getf2_w<T, 4>(pa, batch, st);
        case 2: return launch_getf2_w<T, 2>(pa, batch, st);
    }
    return HARP_E_ARG;
}

template <typename T>
GemmArgs<T> sub_gemm(T* base, int64_t ld, int64_t s, int M, int N, int K, int ar, int ac, int br, int bc, int cr,
                     int cc, T alpha, T beta, const int32_t* active) {
    GemmArgs<T> g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = base + 2 * (size_t(ac) * ld + ar);
    g.lda = ld;
    g.sA = s;
    g.B = base + 2 * (size_t(bc) * ld + br);
    g.ldb = ld;
    g.sB = s;
    g.C = base + 2 * (size_t(cc) * ld + cr);
    g.ldc = ld;
    g.sC = s;
    g.D = const_cast<T*>(g.C);
    g.ldd = ld;
    g.sD = s;
    g.alpha = alpha;
    g.beta = beta;
    g.active = active;
    return g;
}

template <typename T>
harp_status factor_impl(int n, int batch, T* A, int64_t lda, int64_t sA, int32_t* ipiv, int32_t* info, void* blk,
                        hipStream_t st) {
    // Right-looking blocked LU whose trailing update is deferred over NS outer
    // blocks (a super-block of NS * NB columns): within a super-block, an
    // outer block first receives the updates of the earlier outer blocks of
    // the super-block on its own columns (catch-up), is factored, and its row
    // block receives the same updates on the columns to its right (deferred
    // rows) before its block-row solve; the rest of the trailing matrix is
    // updated once per super-block with a contraction of NS * NB.
    constexpr int NB = LuCfg<T>::NB, NS = LuCfg<T>::NS;
    static_assert(NB <= NBMAX, "outer block");
    const Tune tune = tuning_for<T>(n);
    const int W = tune.panel_width;
    HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                     hipLaunchKernelGGL(zero_i32, dim3((batch + 255) / 256), dim3(256), 0, st, info, batch));
    HARP_LAUNCH_CHECK();
    harp_status s;
    for (int K0 = 0; K0 < n; K0 += NS * NB) {
        const int Kend = std::min(n, K0 + NS * NB);
        for (int k0 = K0; k0 < Kend; k0 += NB) {
            const int nbo = std::min(NB, n - k0), kend = k0 + nbo;
            // catch-up: A[k0:n, k0:kend] -= L[k0:n, K0:k0] U[K0:k0, k0:kend]
            if (k0 > K0) {
                GemmArgs<T> g = sub_gemm<T>(A, lda, sA, n - k0, nbo, k0 - K0, k0, K0, K0, k0, k0, k0, T(-1), T(1),
                                            nullptr);
                g.small_grid = tune.small_grid;
                g.site = HARP_SITE_CATCH_UP;
                if ((s = cgemm<T>(g, batch, st)) != HARP_OK) return s;
            }
            // row exchanges reach the block row to the right (then the
            // unit-lower solve and the trailing update) and the earlier
            // columns of the same solve group (so each group's multipliers
            // share one row order)
            const int lbeg = (k0 / kSB) * kSB;
            const bool block_row = kend < n || lbeg < k0;
            for (int j0 = k0; j0 < kend; j0 += W) {
                const int w = std::min(W, kend - j0);
                const bool last = j0 + w == kend;
                PanelArgs pa{A, lda, sA, n, k0, kend, j0, w, ipiv, info, (last && block_row) ? blk : nullptr};
                if ((s = launch_getf2<T>(pa, W, batch, st)) != HARP_OK) return s;
                if (j0 + w < kend) {
                    if ((s = launch_rank_update<T>(A, lda, sA, n, j0, w, kend, batch, st)) != HARP_OK) return s;
                }
            }
            if (block_row) {
                LaswpArgs la{blk, nbo, A, lda, sA, kend, n, lbeg, k0};
                constexpr int CB = LaswpCols<T>::CB;
                const int tiles = (n - kend + CB - 1) / CB + (k0 - lbeg + CB - 1) / CB;
                HARP_PROF_EXT_LAUNCH(HARP_K_TRSM_L, st, 0.0, 0.0, (laswp_kernel<T>), dim3(tiles, batch), dim3(256),
                                     0, la);
                HARP_LAUNCH_CHECK();
            }
            if (kend < n) {
                // deferred rows: A[k0:kend, kend:n] -= L[k0:kend, K0:k0] U[K0:k0, kend:n]
                if (k0 > K0) {
                    GemmArgs<T> g = sub_gemm<T>(A, lda, sA, nbo, n - kend, k0 - K0, k0, K0, K0, kend, k0, kend,
                                                T(-1), T(1), nullptr);
                    g.small_grid = tune.small_grid;
                    g.site = HARP_SITE_DEFERRED_ROWS;
                    if ((s = cgemm<T>(g, batch, st)) != HARP_OK) return s;
                }
                // block row U12 = L11^-1 (exchanged rows), in place: one row
                // tile, so every workgroup reads its whole column block before
                // writing it
                GemmArgs<T> g{};
                g.M = nbo;
                g.N = n - kend;
                g.K = nbo;
                g.A = static_cast<const T*>(blk);
                g.lda = NBMAX;
                g.sA = BlkScratch<T>::stride / int64_t(2 * sizeof(T));
                g.B = A + 2 * (size_t(kend) * lda + k0);
                g.ldb = lda;
                g.sB = sA;
                g.C = nullptr;
                g.ldc = lda;
                g.sC = sA;
                g.D = const_cast<T*>(g.B);
                g.ldd = lda;
                g.sD = sA;
                g.alpha = T(1);
                g.beta = T(0);
                g.active = nullptr;
                g.small_grid = tune.small_grid;
                static_assert(NBMAX <= 64, "the in-place product needs a single row tile");
                g.site = HARP_SITE_BLOCK_ROW;
                if ((s = cgemm<T>(g, batch, st)) != HARP_OK) return s;
            }
        }
        // trailing update of the super-block:
        // A[Kend:n, Kend:n] -= L[Kend:n, K0:Kend] U[K0:Kend, Kend:n]
        if (Kend < n) {
            GemmArgs<T> g = sub_gemm<T>(A, lda, sA, n - Kend, n - Kend, Kend - K0, Kend, K0, K0, Kend, Kend, Kend,
                                        T(-1), T(1), nullptr);
            g.small_grid = tune.small_grid;
            g.site = HARP_SITE_TRAILING;
            if ((s = cgemm<T>(g, batch, st)) != HARP_OK) return s;
        }
    }
    return HARP_OK;
}

// Inverses of the diagonal blocks of every solve group and the groups'
// composite permutations, written into the factor auxiliary buffer.
inline int n_groups(int n) { return (n + kSB - 1) / kSB; }
inline size_t aux_bytes(int n, int batch, int csize) {
    const int64_t G = n_groups(n);
    return size_t(align256(int64_t(batch) * G * kRec * csize) + align256(int64_t(batch) * G * 4 * kSB * 4));
}
template <typename T> inline int32_t* aux_perm(T* aux, int n, int batch) {
    const int64_t G = n_groups(n);
    return reinterpret_cast<int32_t*>(reinterpret_cast<char*>(aux) +
                                      align256(int64_t(batch) * G * kRec * 2 * int64_t(sizeof(T))));
}

template <typename T>
harp_status tri_inverse(int n, int batch, const T* LU, int64_t lda, int64_t sA, const int32_t* ipiv, T* aux,
                        hipStream_t st) {
    const int G = n_groups(n);
    const int small_grid = tuning_for<T>(n).small_grid;
    harp_status s;
    HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                     hipLaunchKernelGGL(group_perm_kernel, dim3(G, batch), dim3(256), 0, st, ipiv, n, G,
                                        aux_perm(aux, n, batch)));
    HARP_LAUNCH_CHECK();
    HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                     hipLaunchKernelGGL((extract_diag_kernel<T>), dim3(G * 16, batch), dim3(256), 0, st, LU, lda, sA,
                                        n, G, aux));
    HARP_LAUNCH_CHECK();
    HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                     hipLaunchKernelGGL((tri_inv16_kernel<T>), dim3(G * batch * (kSB / kInv0), 1, 2), dim3(64), 0,
                                        st, aux, G));
    HARP_LAUNCH_CHECK();
    const int64_t blk = int64_t(kSB) * kSB;
    for (int sz = 2 * kInv0; sz <= kSB; sz *= 2) {
        const int h = sz / 2;
        for (int upper = 0; upper < 2; ++upper) {
            T* M = aux + 2 * (upper ? blk : 0);          // first record's L or U block
            T* tmp = aux + 2 * (2 * blk);                // first record's temp
            // block i of size sz starts at i sz (SB + 1); its quadrants:
            const int64_t q11 = 0, q21 = h, q12 = int64_t(h) * kSB, q22 = int64_t(h) * (kSB + 1);
            GemmArgs<T> g1{}, g2{};
            for (GemmArgs<T>* g : {&g1, &g2}) {
                g->small_grid = small_grid;
                g->M = h;
                g->N = h;
                g->K = h;
                g->beta = T(0);
                g->C = nullptr;
                g->active = nullptr;
                g->inner = kSB / sz;
            }
            // L: tmp = C A^-1, C = -D^-1 tmp ;  U: tmp = B D^-1, B = -A^-1 tmp
            g1.A = M + 2 * (upper ? q12 : q21);
            g1.B = M + 2 * (upper ? q22 : q11);
            g1.D = tmp;
            g2.A = M + 2 * (upper ? q11 : q22);
            g2.B = tmp;
            g2.D = M + 2 * (upper ? q12 : q21);
            g1.lda = g1.ldb = kSB;
            g1.ldd = h;
            g1.ldc = h;
            g2.lda = kSB;
            g2.ldb = h;
            g2.ldd = kSB;
            g2.ldc = kSB;
            g1.alpha = T(1);
            g2.alpha = T(-1);
            g1.sA = g1.sB = g1.sD = kRec;
            g2.sA = g2.sB = g2.sD = kRec;
            g1.sA2 = g1.sB2 = int64_t(sz) * (kSB + 1);
            g1.sD2 = int64_t(h) * h;
            g2.sA2 = g2.sD2 = int64_t(sz) * (kSB + 1);
            g2.sB2 = int64_t(h) * h;
            g1.site = HARP_SITE_TRI_INVERSE;
            if ((s = cgemm<T>(g1, batch * G, st)) != HARP_OK) return s;
            g2.site = HARP_SITE_TRI_INVERSE;
            g2.tri = upper ? 2 : 1;   // A^-1 (upper) or D^-1 (lower): triangular
            if ((s = cgemm<T>(g2, batch * G, st)) != HARP_OK) return s;
        }
    }
    return HARP_OK;
}

// in-place solve of X (n x nrhs, same precision as the factors) by groups of
// SB rows: forward: gather the group's rows through its exchanges, apply the
// inverse unit-lower block, update the rows below; backward: apply the inverse
// upper block, update the rows above.  Tm: SB x nrhs per matrix.
template <typename T>
harp_status solve_impl(int n, int nrhs, int batch, const T* LU, int64_t lda, int64_t sL, const T* aux, T* X,
                       int64_t ldx, int64_t sX, T* Tm, const int32_t* active, int32_t* colnz, hipStream_t st) {
    // colnz (optional, [batch][nrhs]): the forward substitution skips the
    // products of tiles whose right-hand sides are exactly zero in the
    // group's rows (the diagonal block's product then stores zeros, the
    // update leaves the rows below as they are).  The solution of L Y = P B is zero above the first non-zero row
    // of each column of P B, so right-hand sides that start low (port
    // excitations touch only their own antenna's rows) leave most of the
    // early groups' updates out.
    const int G = n_groups(n);
    const int64_t sT = int64_t(kSB) * nrhs;
    const int32_t* perm = aux_perm(const_cast<T*>(aux), n, batch);
    const int64_t blk = int64_t(kSB) * kSB;
    const int small_grid = tuning_for<T>(n).small_grid;
    harp_status s;
    auto gemm = [&](int site, int M, int N, int K, const T* A, int64_t lda_, int64_t sA_, const T* B, int64_t ldb_,
                    int64_t sB_, T* D, int64_t ldd_, int64_t sD_, T alpha, T beta, int tri = 0,
                    const int32_t* b_nz = nullptr) {
        GemmArgs<T> g{};
        g.tri = tri;
        g.b_nz = b_nz;
        g.s_nz = nrhs;
        g.M = M;
        g.N = N;
        g.K = K;
        g.A = A;
        g.lda = lda_;
        g.sA = sA_;
        g.B = B;
        g.ldb = ldb_;
        g.sB = sB_;
        g.C = beta != T(0) ? D : nullptr;
        g.ldc = ldd_;
        g.sC = sD_;
        g.D = D;
        g.ldd = ldd_;
        g.sD = sD_;
        g.alpha = alpha;
        g.beta = beta;
        g.active = active;
        g.site = site;
        // with zero-column skipping, 32-column tiles: a tile's right-hand
        // sides then start in the same 256-row group more often (32 ports of
        // 8 rows), and the tiles left to run spread over more workgroups
        g.small_grid = b_nz ? INT_MAX : small_grid;
        return cgemm<T>(g, batch, st);
    };
    for (int gi = 0; gi < G; ++gi) {
        const int g0 = gi * kSB, sb = std::min(kSB, n - g0), gend = g0 + sb;
        HARP_PROF_LAUNCH(HARP_K_TRSM_L, st, 0.0, 0.0,
                         hipLaunchKernelGGL((group_gather_kernel<T>),
                                            dim3((nrhs + kGatherCols - 1) / kGatherCols, batch), dim3(256), 0, st,
                                            perm, G, gi, sb, X, ldx, sX, nrhs, Tm, sT, active, colnz));
        HARP_LAUNCH_CHECK();
        const T* Linv = aux + 2 * (int64_t(gi) * kRec);
        // the inverse blocks are exactly triangular: their zero halves are skipped
        if ((s = gemm(HARP_SITE_SOLVE_DIAG, sb, nrhs, sb, Linv, kSB, G * kRec, Tm, kSB, sT, X + 2 * size_t(g0), ldx, sX,
                      T(1), T(0), 1, colnz)) != HARP_OK)
            return s;
        if (gend < n &&
            (s = gemm(HARP_SITE_SOLVE_UPDATE, n - gend, nrhs, sb, LU + 2 * (size_t(g0) * lda + gend), lda, sL, X + 2 * size_t(g0), ldx, sX,
                      X + 2 * size_t(gend), ldx, sX, T(-1), T(1), 0, colnz)) != HARP_OK)
            return s;
    }
    for (int gi = G - 1; gi >= 0; --gi) {
        const int g0 = gi * kSB, sb = std::min(kSB, n - g0);
        const T* Uinv = aux + 2 * (int64_t(gi) * kRec + blk);
        if ((s = gemm(HARP_SITE_SOLVE_DIAG, sb, nrhs, sb, Uinv, kSB, G * kRec, X + 2 * size_t(g0), ldx, sX, Tm, kSB, sT,
                      T(1), T(0), 2)) != HARP_OK)
            return s;
        if (g0 > 0 && (s = gemm(HARP_SITE_SOLVE_UPDATE, g0, nrhs, sb, LU + 2 * (size_t(g0) * lda), lda, sL, Tm, kSB, sT, X, ldx, sX, T(-1),
                                T(1))) != HARP_OK)
            return s;
        // copy the group's solution back
        using V = typename C2<T>::t;
        const int64_t total = int64_t(sb) * nrhs;
        const unsigned blocks = unsigned(std::min<int64_t>((total + 255) / 256, 1024));
        HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                         hipLaunchKernelGGL((convert_kernel<V, V>), dim3(blocks, 1, batch), dim3(256), 0, st,
                                            reinterpret_cast<const V*>(Tm), int64_t(kSB), sT,
                                            reinterpret_cast<V*>(X) + g0, ldx, sX, sb, nrhs, active));
        HARP_LAUNCH_CHECK();
    }
    return HARP_OK;
}

template <typename Ti, typename To>
harp_status convert(const void* src, int64_t lds, int64_t ss, void* dst, int64_t ldd, int64_t sd, int rows, int cols,
                    int batch, const int32_t* active, hipStream_t st) {
    const int64_t total = int64_t(rows) * cols;
    const unsigned blocks = unsigned(std::min<int64_t>((total + 255) / 256, 2048));
    HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                     hipLaunchKernelGGL((convert_kernel<Ti, To>), dim3(blocks, 1, batch), dim3(256), 0, st,
                                        static_cast<const Ti*>(src), lds, ss, static_cast<To*>(dst), ldd, sd, rows,
                                        cols, active));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

// Frobenius norms of `batch` complex128 matrices into out[batch]
// (complex64: M holds complex64 values, squared in FP64)
harp_status fro_norms(const void* M, bool complex64, int64_t ld, int64_t s, int rows, int cols, int batch,
                      double* part, double* out, hipStream_t st) {
    int nblk = norm_blocks(rows, cols);
    if (complex64) {
        nblk = norm_blocks((rows + 1) / 2, cols);   // units of 256 row pairs
        const bool vec2 = rows % 2 == 0 && ld % 2 == 0 && (batch == 1 || s % 2 == 0) &&
                          (reinterpret_cast<uintptr_t>(M) & 15) == 0;
        HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                         hipLaunchKernelGGL(sumsq_partial_c64_kernel, dim3(nblk, 1, batch), dim3(256), 0, st,
                                            static_cast<const float2*>(M), ld, s, rows, cols, vec2, part, 0,
                                            static_cast<const int32_t*>(nullptr)));
    } else
        HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                         hipLaunchKernelGGL(sumsq_partial_kernel, dim3(nblk, 1, batch), dim3(256), 0, st,
                                            static_cast<const double2*>(M), ld, s,
                                            static_cast<const double2*>(nullptr), int64_t(0), int64_t(0), rows,
                                            cols, part, static_cast<const int32_t*>(nullptr)));
    HARP_LAUNCH_CHECK();
    HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                     hipLaunchKernelGGL(sumsq_final_kernel, dim3(batch), dim3(256), 0, st, part, out, nblk));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

// The residual after a correction, with complex64 factors and a complex64
// matrix, is updated as R - Z D (D the complex64 correction just added to X):
// Z D in res_slices(n) products over consecutive K slices of res_slice_k(n)
// (the last one shorter), each on the FP32 matrix cores, the slices added in
// FP64.  Each slice's products are accumulated in FP32 over at most
// res_slice_k(n) complex terms, which bounds their error (residual_bound).
constexpr int kResSlicesMax = 16;
inline int res_slices(int n) { return std::max(1, std::min(kResSlicesMax, (n + 255) / 256)); }
inline int res_slice_k(int n) {
    const int S = res_slices(n), ks = (n + S - 1) / S;
    return (ks + 15) / 16 * 16;
}
inline int res_slice_count(int n) { return (n + res_slice_k(n) - 1) / res_slice_k(n); }

struct SolveWs {
    float2* B32;      // n x nrhs complex64 per matrix (ld n)
    double2* R;       // n x nrhs complex128 per matrix (ld n)
    void* Tm;         // SB x nrhs per matrix in the factor precision (group temp)
    float2* P;        // [batch][res_slice_count(n)] n x nrhs complex64: slices of Z D
    double* bnd;      // [batch]: running error bound of the updated residual
    double* part;     // [batch][kNormSlots][kNormBlocks]
    double* znorm;    // [batch]: ||Z||_F
    int32_t* active;  // [batch]
    harp_refine_report* rep;   // [batch]
    int32_t* colnz;   // [batch][nrhs]: non-zero columns of a group's right-hand sides (first solve)
};

size_t solve_ws_layout(int n, int nrhs, int batch, int dtype, int refine, SolveWs* w, char* base) {
    const int64_t mat = int64_t(n) * nrhs;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off += align256(bytes);
        return base ? base + o : nullptr;
    };
    SolveWs tmp{};
    SolveWs& W = w ? *w : tmp;
    W.B32 = reinterpret_cast<float2*>(take((dtype == HARP_C64) ? mat * batch * 8 : 0));
    W.R = reinterpret_cast<double2*>(take(refine ? mat * batch * 16 : 0));
    W.Tm = take(int64_t(kSB) * nrhs * batch * (dtype == HARP_C64 ? 8 : 16));
    const bool upd = refine && dtype == HARP_C64;
    W.P = reinterpret_cast<float2*>(take(upd ? int64_t(res_slice_count(n)) * mat * batch * 8 : 0));
    W.bnd = reinterpret_cast<double*>(take(refine ? int64_t(batch) * 8 : 0));
    W.part = reinterpret_cast<double*>(take(refine ? int64_t(batch) * kNormSlots * kNormBlocks * 8 : 0));
    W.znorm = reinterpret_cast<double*>(take(refine ? int64_t(batch) * 8 : 0));
    W.active = reinterpret_cast<int32_t*>(take(refine ? int64_t(batch) * 4 : 0));
    W.rep = reinterpret_cast<harp_refine_report*>(take(refine ? int64_t(batch) * int64_t(sizeof(harp_refine_report)) : 0));
    W.colnz = reinterpret_cast<int32_t*>(take(int64_t(batch) * nrhs * 4));
    return size_t(off);
}

}  // namespace
}  // namespace harp

using namespace harp;

extern "C" harp_status harp_set_tuning(const harp_tuning_entry* entries, int32_t n_entries) {
    if (n_entries < 0 || n_entries > kMaxTuning || (n_entries > 0 && !entries)) return HARP_E_ARG;
    for (int i = 0; i < n_entries; ++i) {
        const harp_tuning_entry& e = entries[i];
        if (e.max_order <= 0 || e.max_order > 8192 || (i > 0 && e.max_order <= entries[i - 1].max_order))
            return HARP_E_ARG;
        if (!panel_feasible<float>(e.panel_width_c64, e.max_order) ||
            !panel_feasible<double>(e.panel_width_c128, e.max_order))
            return HARP_E_ARG;
        if (e.small_grid_wgs < 0) return HARP_E_ARG;
    }
    std::lock_guard<std::mutex> lock(g_tuning_mutex);
    for (int i = 0; i < n_entries; ++i) g_tuning[i] = entries[i];
    g_n_tuning = n_entries;
    return HARP_OK;
}

extern "C" harp_status harp_get_tuning(harp_tuning_entry* entries, int32_t capacity, int32_t* n_entries) {
    if (!n_entries || capacity < 0 || (capacity > 0 && !entries)) return HARP_E_ARG;
    std::lock_guard<std::mutex> lock(g_tuning_mutex);
    *n_entries = g_n_tuning;
    for (int i = 0; i < g_n_tuning && i < capacity; ++i) entries[i] = g_tuning[i];
    return HARP_OK;
}

extern "C" harp_status harp_default_tuning(int32_t n, harp_tuning_entry* entry) {
    if (!entry || n <= 0 || n > 8192) return HARP_E_ARG;
    entry->max_order = n;
    entry->panel_width_c64 = default_panel_width<float>(n);
    entry->panel_width_c128 = default_panel_width<double>(n);
    entry->small_grid_wgs = 1024;
    return HARP_OK;
}

extern "C" harp_status reduced_factor_ws(int32_t n, int32_t batch, harp_dtype dtype, size_t* bytes) {
    if (!bytes || n <= 0 || batch <= 0 || (dtype != HARP_C64 && dtype != HARP_C128)) return HARP_E_ARG;
    *bytes = aux_bytes(n, batch, dtype == HARP_C64 ? 8 : 16);
    return HARP_OK;
}

extern "C" harp_status reduced_factor(int32_t n, int32_t batch, harp_dtype dtype, void* d_A, int64_t lda,
                                      int64_t stride_a, int32_t* d_ipiv, int32_t* d_info, void* d_aux,
                                      size_t aux_size, hipStream_t stream) {
    if (!d_A || !d_ipiv || !d_info || n <= 0 || batch <= 0) return HARP_E_ARG;
    if (n > 8192) return HARP_E_ARG;
    if (lda < n || (batch > 1 && stride_a < lda * n)) return HARP_E_ARG;
    if (dtype != HARP_C64 && dtype != HARP_C128) return HARP_E_ARG;
    if (int64_t(batch) * n_groups(n) * (kSB / kInv0) > 65535 || batch > 65535) return HARP_E_ARG;
    if (!d_aux || aux_size < aux_bytes(n, batch, dtype == HARP_C64 ? 8 : 16)) return HARP_E_WORKSPACE;
    harp_status s;
    if (dtype == HARP_C64) {
        float* A = static_cast<float*>(d_A);
        if ((s = factor_impl<float>(n, batch, A, lda, stride_a, d_ipiv, d_info, d_aux, stream)) != HARP_OK) return s;
        return tri_inverse<float>(n, batch, A, lda, stride_a, d_ipiv, static_cast<float*>(d_aux), stream);
    }
    double* A = static_cast<double*>(d_A);
    if ((s = factor_impl<double>(n, batch, A, lda, stride_a, d_ipiv, d_info, d_aux, stream)) != HARP_OK) return s;
    return tri_inverse<double>(n, batch, A, lda, stride_a, d_ipiv, static_cast<double*>(d_aux), stream);
}

extern "C" harp_status reduced_solve_ws(int32_t n, int32_t nrhs, int32_t batch, harp_dtype dtype, int32_t refine,
                                        size_t* bytes) {
    if (!bytes || n <= 0 || nrhs <= 0 || batch <= 0 || (dtype != HARP_C64 && dtype != HARP_C128)) return HARP_E_ARG;
    *bytes = solve_ws_layout(n, nrhs, batch, dtype, refine, nullptr, nullptr);
    return HARP_OK;
}

namespace harp {
namespace {

// The solve with its workspace at d_ws (ws_bytes; the caller's, or the
// library's static scratch).
harp_status solve_core(int32_t n, int32_t nrhs, int32_t batch, harp_dtype dtype, const void* d_LU, int64_t lda,
                       int64_t stride_lu, const int32_t* d_ipiv, const void* d_aux, size_t aux_size,
                       const void* d_B, int64_t ldb, int64_t stride_b, void* d_X, int64_t ldx, int64_t stride_x,
                       const harp_refine* refine, harp_refine_report* report, void* d_ws, size_t ws_bytes,
                       hipStream_t st) {
    if (!d_LU || !d_ipiv || !d_B || !d_X || n <= 0 || nrhs <= 0 || batch <= 0 || batch > 65535) return HARP_E_ARG;
    if (dtype != HARP_C64 && dtype != HARP_C128) return HARP_E_ARG;
    if (!d_aux || aux_size < aux_bytes(n, batch, dtype == HARP_C64 ? 8 : 16)) return HARP_E_WORKSPACE;
    if (lda < n || ldb < n || ldx < n) return HARP_E_ARG;
    if (batch > 1 && (stride_lu < lda * n || stride_b < ldb * nrhs || stride_x < ldx * nrhs)) return HARP_E_ARG;
    const bool ref = refine != nullptr;
    if (ref) {
        if (!refine->d_Z || refine->ldz < n || refine->max_iter < 0 || !(refine->tol >= 0.0)) return HARP_E_ARG;
        if (refine->z_complex64 != 0 && refine->z_complex64 != 1) return HARP_E_ARG;
        if (batch > 1 && refine->stride_z < refine->ldz * n) return HARP_E_ARG;
    }
    const size_t need = solve_ws_layout(n, nrhs, batch, dtype, ref, nullptr, nullptr);
    if (need > 0 && (!d_ws || ws_bytes < need)) return HARP_E_WORKSPACE;
    SolveWs W{};
    solve_ws_layout(n, nrhs, batch, dtype, ref, &W, static_cast<char*>(d_ws));
    const int64_t mat = int64_t(n) * nrhs;
    harp_status s;

    // solve in the factor precision; the result is written into X, or added
    // to X (corrections)
    auto solve_into = [&](const void* rhs, int64_t ldr, int64_t sr, const int32_t* act,
                          bool accumulate) -> harp_status {
        harp_status q;
        double2* Xd = static_cast<double2*>(d_X);
        const unsigned blocks = unsigned(std::min<int64_t>((mat + 255) / 256, 2048));
        if (dtype == HARP_C64) {
            const float* LU = static_cast<const float*>(d_LU);
            if ((q = convert<double2, float2>(rhs, ldr, sr, W.B32, n, mat, n, nrhs, batch, act, st)) != HARP_OK)
                return q;
            if ((q = solve_impl<float>(n, nrhs, batch, LU, lda, stride_lu, static_cast<const float*>(d_aux),
                                       reinterpret_cast<float*>(W.B32), n, mat, static_cast<float*>(W.Tm), act,
                                       accumulate ? nullptr : W.colnz, st)) != HARP_OK)
                return q;
            if (accumulate) {
                HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                                 hipLaunchKernelGGL(axpy_kernel<float2>, dim3(blocks, 1, batch), dim3(256), 0, st, Xd,
                                                    ldx, stride_x, W.B32, n, mat, n, nrhs, act));
                HARP_LAUNCH_CHECK();
                return HARP_OK;
            }
            return convert<float2, double2>(W.B32, n, mat, Xd, ldx, stride_x, n, nrhs, batch, act, st);
        }
        const double* LU = static_cast<const double*>(d_LU);
        if (accumulate) {   // rhs is the residual W.R: solve it in place, then add
            if ((q = solve_impl<double>(n, nrhs, batch, LU, lda, stride_lu, static_cast<const double*>(d_aux),
                                        reinterpret_cast<double*>(W.R), n, mat, static_cast<double*>(W.Tm), act,
                                        nullptr, st)) != HARP_OK)
                return q;
            HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                             hipLaunchKernelGGL(axpy_kernel<double2>, dim3(blocks, 1, batch), dim3(256), 0, st, Xd,
                                                ldx, stride_x, W.R, n, mat, n, nrhs, act));
            HARP_LAUNCH_CHECK();
            return HARP_OK;
        }
        if ((q = convert<double2, double2>(rhs, ldr, sr, Xd, ldx, stride_x, n, nrhs, batch, act, st)) != HARP_OK)
            return q;
        return solve_impl<double>(n, nrhs, batch, LU, lda, stride_lu, static_cast<const double*>(d_aux),
                                  reinterpret_cast<double*>(Xd), ldx, stride_x, static_cast<double*>(W.Tm), act,
                                  W.colnz, st);
    };

    if ((s = solve_into(d_B, ldb, stride_b, nullptr, false)) != HARP_OK) return s;
    if (!ref) return HARP_OK;

    // FP64 iterative refinement, controlled on the device: each round takes
    // the FP64 residual of the active systems, its norm and the check kernel,
    // then (unless it is the last round) the correction solve.  With a host
    // report the host looks at the active flags only from the second round
    // on (the complex64 solve alone never meets an FP64 tolerance), so a
    // system that converges after one correction costs a single
    // synchronisation; without one nothing synchronises and the whole sweep
    // budget is enqueued.
    harp_refine_report* rep = refine->d_report ? static_cast<harp_refine_report*>(refine->d_report) : W.rep;
    const bool host = report != nullptr;
    const unsigned gb = unsigned((batch + 63) / 64);
    const int rnblk = norm_blocks(n, nrhs);   // blocks per matrix of the residual and solution norms
    HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                     hipLaunchKernelGGL(refine_init_kernel, dim3(gb), dim3(64), 0, st, W.active, rep, W.bnd, batch));
    HARP_LAUNCH_CHECK();
    const bool z32 = refine->z_complex64 != 0;
    if ((s = fro_norms(refine->d_Z, z32, refine->ldz, refine->stride_z, n, n, batch, W.part, W.znorm, st)) !=
        HARP_OK)
        return s;
    int n_act = batch;   // systems the host knows to be active (work accounting of the timers only)
    // error bound of a residual update R - Z D (complex64 Z and D, products
    // accumulated in FP32 over at most Ks complex terms per slice, slices
    // added in FP64): per element sqrt(2) gamma_{2 Ks + 2} (|Z| |D|), so in
    // the Frobenius norm bc ||Z||_F ||D||_F, plus the FP64 rounding of X + D
    // (u64 ||Z||_F ||X||_F) and terms flushed below the FP32 normal range
    // (babs)
    const int Ks = res_slice_k(n), n_sl = res_slice_count(n), full_sl = n / Ks, tail_k = n - full_sl * Ks;
    const double u32 = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
    const double m_terms = 2.0 * Ks + 2.0;
    const double bc = 1.01 * std::sqrt(2.0) * m_terms * u32 / (1.0 - m_terms * u32);
    const double babs = std::sqrt(2.0) * (2.0 * n + 2.0 * n_sl) * std::ldexp(1.0, -126) * std::sqrt(double(n) * nrhs);
    const int dnblk = norm_blocks((n + 1) / 2, nrhs);
    const bool dvec2 = n % 2 == 0 && (reinterpret_cast<uintptr_t>(W.B32) & 15) == 0;
    for (int it = 0;; ++it) {
        // the first residual after a correction is updated; any later one is
        // a full FP64 residual again (which resets the bound), so a tolerance
        // below the update's bound still converges, one sweep later
        const bool update = it == 1 && z32 && W.P != nullptr;
        if (!update) {
            // R = B - Z X  (FP64, MFMA)
            GemmArgs<double> g;
            g.M = n;
            g.N = nrhs;
            g.K = n;
            // complex64 Z: widened to FP64 as the residual product loads it
            g.A = z32 ? nullptr : static_cast<const double*>(refine->d_Z);
            g.A32 = z32 ? static_cast<const float*>(refine->d_Z) : nullptr;
            g.lda = refine->ldz;
            g.sA = refine->stride_z;
            g.B = static_cast<const double*>(d_X);
            g.ldb = ldx;
            g.sB = stride_x;
            g.C = static_cast<const double*>(d_B);
            g.ldc = ldb;
            g.sC = stride_b;
            g.D = reinterpret_cast<double*>(W.R);
            g.ldd = n;
            g.sD = mat;
            g.alpha = -1.0;
            g.beta = 1.0;
            g.active = W.active;
            g.site = HARP_SITE_RESIDUAL;
            if ((s = cgemm<double>(g, batch, st, n_act)) != HARP_OK) return s;
        } else {
            // R = R - Z D with D (W.B32) the complex64 correction the last
            // sweep added to X: slice q of Z D (K range [q Ks, q Ks + Ks))
            // into P[q], then the slices subtracted in FP64
            GemmArgs<float> g{};
            g.M = n;
            g.N = nrhs;
            g.K = Ks;
            g.A = static_cast<const float*>(refine->d_Z);
            g.lda = refine->ldz;
            g.sA = refine->stride_z;
            g.sA2 = int64_t(Ks) * refine->ldz;
            g.B = reinterpret_cast<const float*>(W.B32);
            g.ldb = n;
            g.sB = mat;
            g.sB2 = Ks;
            g.C = nullptr;
            g.D = reinterpret_cast<float*>(W.P);
            g.ldd = n;
            g.sD = int64_t(n_sl) * mat;
            g.sD2 = mat;
            g.alpha = 1.0f;
            g.beta = 0.0f;
            g.active = W.active;
            g.site = HARP_SITE_RESIDUAL_UPDATE;
            g.inner = full_sl;
            if (full_sl > 0 && (s = cgemm<float>(g, batch, st, n_act)) != HARP_OK) return s;
            if (tail_k > 0) {
                g.inner = 1;
                g.K = tail_k;
                g.A += 2 * size_t(full_sl) * Ks * refine->ldz;
                g.B += 2 * size_t(full_sl) * Ks;
                g.D += 2 * size_t(full_sl) * mat;
                g.sA2 = g.sB2 = g.sD2 = 0;
                if ((s = cgemm<float>(g, batch, st, n_act)) != HARP_OK) return s;
            }
            const unsigned ub = unsigned(std::min<int64_t>((mat + 255) / 256, 2048));
            HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                             hipLaunchKernelGGL(residual_update_kernel, dim3(ub, 1, batch), dim3(256), 0, st, W.R,
                                                int64_t(n), mat, static_cast<const float2*>(W.P), mat,
                                                int64_t(n_sl) * mat, n_sl, n, nrhs,
                                                static_cast<const int32_t*>(W.active)));
            HARP_LAUNCH_CHECK();
            HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                             hipLaunchKernelGGL(sumsq_partial_c64_kernel, dim3(dnblk, 1, batch), dim3(256), 0, st,
                                                static_cast<const float2*>(W.B32), int64_t(n), mat, n, nrhs, dvec2,
                                                W.part, 2, static_cast<const int32_t*>(W.active)));
            HARP_LAUNCH_CHECK();
        }
        HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                         hipLaunchKernelGGL(sumsq_partial_kernel, dim3(rnblk, 2, batch), dim3(256), 0, st,
                                            static_cast<const double2*>(W.R), int64_t(n), mat,
                                            static_cast<const double2*>(d_X), ldx, stride_x, n, nrhs, W.part,
                                            static_cast<const int32_t*>(W.active)));
        HARP_LAUNCH_CHECK();
        HARP_PROF_LAUNCH(HARP_K_AUX, st, 0.0, 0.0,
                         hipLaunchKernelGGL(refine_check_kernel, dim3(batch), dim3(256), 0, st, W.part, rnblk,
                                            update ? dnblk : 0, W.znorm, refine->tol, refine->max_iter, bc,
                                            babs, u64, W.bnd, W.active, rep));
        HARP_LAUNCH_CHECK();
        if (it == refine->max_iter) break;
        if (host && it >= 1) {
            // a system is still active after check `it` exactly when its
            // iteration count is it + 1 (every check of an active system
            // counts one correction), so the report alone tells the host
            HARP_HIP_CHECK(hipMemcpyAsync(report, rep, sizeof(harp_refine_report) * batch, hipMemcpyDeviceToHost,
                                          st));
            HARP_HIP_CHECK(hipStreamSynchronize(st));
            n_act = 0;
            for (int b = 0; b < batch; ++b) n_act += report[b].iters == it + 1;
            if (n_act == 0) break;
        }
        // correction: D = LU^-1 R, X += D (inactive systems skip every kernel)
        if ((s = solve_into(W.R, n, mat, W.active, true)) != HARP_OK) return s;
    }
    if (!host) return HARP_OK;
    HARP_HIP_CHECK(hipMemcpyAsync(report, rep, sizeof(harp_refine_report) * batch, hipMemcpyDeviceToHost, st));
    HARP_HIP_CHECK(hipStreamSynchronize(st));
    for (int b = 0; b < batch; ++b)
        if (!report[b].converged) return HARP_E_NOCONV;
    return HARP_OK;
}

// Static scratch of reduced_solve_noalloc: a file-scope device array, one
// copy per GPU, allocated with the code object and held until the process
// ends.  Host code never passes `scratch` itself (on the host it is only a
// stand-in symbol): its device address comes from hipGetSymbolAddress, once
// per device, with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

harp_status scratch_for_current_device(void** out) {
    int dev = -1;
    HARP_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return HARP_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HARP_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HARP_OK;
}

}  // namespace
}  // namespace harp

extern "C" harp_status reduced_solve(int32_t n, int32_t nrhs, int32_t batch, harp_dtype dtype, const void* d_LU,
                                     int64_t lda, int64_t stride_lu, const int32_t* d_ipiv, const void* d_aux,
                                     size_t aux_size, const void* d_B, int64_t ldb, int64_t stride_b, void* d_X,
                                     int64_t ldx, int64_t stride_x, const harp_refine* refine,
                                     harp_refine_report* report, void* d_ws, size_t ws_bytes, hipStream_t st) {
    return solve_core(n, nrhs, batch, dtype, d_LU, lda, stride_lu, d_ipiv, d_aux, aux_size, d_B, ldb, stride_b, d_X,
                      ldx, stride_x, refine, report, d_ws, ws_bytes, st);
}

extern "C" size_t reduced_solve_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" harp_status reduced_solve_noalloc(int32_t n, int32_t nrhs, int32_t batch, harp_dtype dtype,
                                             const void* d_LU, int64_t lda, int64_t stride_lu, const int32_t* d_ipiv,
                                             const void* d_aux, size_t aux_size, const void* d_B, int64_t ldb,
                                             int64_t stride_b, void* d_X, int64_t ldx, int64_t stride_x,
                                             const harp_refine* refine, harp_refine_report* report, hipStream_t st) {
    if (n <= 0 || nrhs <= 0 || batch <= 0 || (dtype != HARP_C64 && dtype != HARP_C128)) return HARP_E_ARG;
    const size_t need = solve_ws_layout(n, nrhs, batch, dtype, refine != nullptr, nullptr, nullptr);
    if (need > kScratchBytes) return HARP_E_WORKSPACE;
    void* ws = nullptr;
    harp_status s = scratch_for_current_device(&ws);
    if (s != HARP_OK) return s;
    return solve_core(n, nrhs, batch, dtype, d_LU, lda, stride_lu, d_ipiv, d_aux, aux_size, d_B, ldb, stride_b, d_X,
                      ldx, stride_x, refine, report, ws, kScratchBytes, st);
}

#include "../../include/harp_debug.h"

extern "C" harp_status harp_debug_cgemm(harp_dtype dtype, int32_t M, int32_t N, int32_t K, int32_t batch, double alpha,
                                        const void* d_A, int64_t lda, int64_t sA, const void* d_B, int64_t ldb,
                                        int64_t sB, double beta, const void* d_C, int64_t ldc, int64_t sC, void* d_D,
                                        int64_t ldd, int64_t sD, hipStream_t stream) {
    return harp_cgemm(dtype, M, N, K, batch, alpha, d_A, lda, sA, d_B, ldb, sB, beta, d_C, ldc, sC, d_D, ldd, sD,
                      stream);
}

extern "C" harp_status harp_cgemm(harp_dtype dtype, int32_t M, int32_t N, int32_t K, int32_t batch, double alpha,
                                  const void* d_A, int64_t lda, int64_t sA, const void* d_B, int64_t ldb, int64_t sB,
                                  double beta, const void* d_C, int64_t ldc, int64_t sC, void* d_D, int64_t ldd,
                                  int64_t sD, hipStream_t stream) {
    if (M < 0 || N < 0 || K < 0 || batch <= 0 || batch > 65535 || !d_D) return HARP_E_ARG;
    if ((K > 0 && (!d_A || !d_B)) || (beta != 0.0 && !d_C)) return HARP_E_ARG;
    if (lda < std::max(1, M) || ldb < std::max(1, K) || ldd < std::max(1, M)) return HARP_E_ARG;
    if (beta != 0.0 && ldc < std::max(1, M)) return HARP_E_ARG;
    if (dtype == HARP_C64) {
        GemmArgs<float> g{M, N, K, static_cast<const float*>(d_A), lda, sA, static_cast<const float*>(d_B), ldb, sB,
                          static_cast<const float*>(d_C), ldc, sC, static_cast<float*>(d_D), ldd, sD,
                          float(alpha), float(beta), nullptr};
        return cgemm<float>(g, batch, stream);
    }
    if (dtype == HARP_C128) {
        GemmArgs<double> g{M, N, K, static_cast<const double*>(d_A), lda, sA, static_cast<const double*>(d_B), ldb, sB,
                           static_cast<const double*>(d_C), ldc, sC, static_cast<double*>(d_D), ldd, sD, alpha, beta,
                           nullptr};
        return cgemm<double>(g, batch, stream);
    }
    return HARP_E_ARG;
}
