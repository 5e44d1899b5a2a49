// Adjoint (vector-Jacobian products) of the fill and of the port step with
// respect to the antenna positions, for array synthesis.
//
// Conventions: for a real objective J of complex outputs, a cotangent G of an
// output Z is the array with dJ = Re sum conj(G) dZ (the convention of
// PyTorch's complex autograd).  The fill's product takes instead the array
// Wz = conj(G) directly: gx_i += Re sum_ab Wz_ab dZ_ab / dx_i.
//
// Fill (Eq. 4).  For the pair (m, n), R = p_m - p_n, r = |R|, alpha the angle
// of R, t = r_min / r, w = e^{j alpha}:
//   Z_TS = e^{-jkr} w^{-P} A,   A = sum_{p'=0..2P} w^{p'} H_{p'-P}(t),
//   dZ/dr     = -jk Z + e^{-jkr} w^{-P} A_t (-t / r),   A_t = sum w^{p'} H'_{p'-P}(t)
//   dZ/dalpha = j e^{-jkr} w^{-P} (A_p - P A),          A_p = sum p' w^{p'} H_{p'-P}(t)
//   dZ/dR_x = cos(alpha) dZ/dr - sin(alpha)/r dZ/dalpha
//   dZ/dR_y = sin(alpha) dZ/dr + cos(alpha)/r dZ/dalpha
// (H, H' by Horner in t with its derivative; A and w dA/dw by Horner in w with
// its derivative).  Since dR/dp_m = I and dR/dp_n = -I, the pair adds
// c = Re sum_TS Wz[(m,T),(n,S)] dZ_TS/dR to the gradient of m and subtracts it
// from that of n.  Self blocks do not depend on positions; blocks beyond the
// radius of influence are constant zero.
//
// Mapping as in the fill (64 testing antennas on the lanes x 16 source
// antennas per 256-thread workgroup); per-antenna sums are reduced in a fixed
// order (lanes, then waves, then tiles), so the result is deterministic.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "prof.hpp"

namespace harp {
namespace {

constexpr int kTM = 64;   // testing antennas per workgroup (lanes)
constexpr int kGA = 4;    // source antennas per thread
constexpr int kTN = 4 * kGA;

struct VjpArgs {
    const char* model;
    const double* x;
    const double* y;
    int n_ant, n_mbf;
    double ri;
    const double2* W;      // Wz, n x n column-major
    int64_t ldw;
    double* part_m;        // [tiles_n][n_ant][2]: sums over a tile's source antennas
    double* part_n;        // [tiles_m][n_ant][2]: sums over a tile's testing antennas
    int32_t* info;         // set to -1 when the model does not match (n_mbf, Q)
};

template <int Q>
__global__ void __launch_bounds__(256) fill_vjp_kernel(VjpArgs a, const double* __restrict__ coef) {
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(a.model);
    if (h->magic != kModelMagic || h->n_mbf != a.n_mbf || h->Q != Q || h->P < 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(a.info, -1);
        return;
    }
    const int P = h->P, nm = a.n_mbf, np = 2 * P + 1;
    const double k = h->k, r_min = h->r_min;
    const int tiles_m = (a.n_ant + kTM - 1) / kTM;
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int m = tm * kTM + lane;

    bool live[kGA];
    double t[kGA], ir[kGA], ca[kGA], sa[kGA];
    cpx<double> w[kGA], ph[kGA];
    const double xm = m < a.n_ant ? a.x[m] : 0.0, ym = m < a.n_ant ? a.y[m] : 0.0;
#pragma unroll
    for (int g = 0; g < kGA; ++g) {
        const int n = tn * kTN + wave * kGA + g;
        live[g] = false;
        t[g] = ir[g] = ca[g] = sa[g] = 0.0;
        w[g] = {1.0, 0.0};
        ph[g] = {0.0, 0.0};
        if (m >= a.n_ant || n >= a.n_ant || m == n) continue;
        const double dx = xm - a.x[n], dy = ym - a.y[n];
        const double r = sqrt(dx * dx + dy * dy);
        if (a.ri > 0.0 && r > a.ri) continue;
        live[g] = true;
        ir[g] = 1.0 / r;
        t[g] = r_min * ir[g];
        ca[g] = dx * ir[g];
        sa[g] = dy * ir[g];
        w[g] = {ca[g], sa[g]};
        double th = -k * r - double(P) * atan2(dy, dx);
        th -= kTwoPi * rint(th * (1.0 / kTwoPi));
        double s, c;
        sincos(th, &s, &c);
        ph[g] = {c, s};
    }
    bool any = false;
#pragma unroll
    for (int g = 0; g < kGA; ++g) any |= live[g];
    const bool wave_live = __ballot(any) != 0;

    double cx[kGA], cy[kGA];
#pragma unroll
    for (int g = 0; g < kGA; ++g) cx[g] = cy[g] = 0.0;

    if (wave_live) {
        for (int S = 0; S < nm; ++S) {
            for (int T = 0; T < nm; ++T) {
                const double* cts = coef + size_t(T * nm + S) * np * (Q + 1) * 2;
                // Horner in w (with derivative) over p' = 2P..0 of H and H'
                cpx<double> A[kGA], Ad[kGA], At[kGA];
#pragma unroll
                for (int g = 0; g < kGA; ++g) A[g] = Ad[g] = At[g] = {0.0, 0.0};
                for (int pp = np - 1; pp >= 0; --pp) {
                    const double* cq = cts + pp * (Q + 1) * 2;
                    double cr[Q + 1], ci[Q + 1];
#pragma unroll
                    for (int q = 0; q <= Q; ++q) {
                        cr[q] = cq[2 * q];
                        ci[q] = cq[2 * q + 1];
                    }
#pragma unroll
                    for (int g = 0; g < kGA; ++g) {
                        // H(t) and H'(t)
                        double hr = cr[Q], hi = ci[Q], dr = 0.0, di = 0.0;
#pragma unroll
                        for (int q = Q - 1; q >= 0; --q) {
                            dr = fma(dr, t[g], hr);
                            di = fma(di, t[g], hi);
                            hr = fma(hr, t[g], cr[q]);
                            hi = fma(hi, t[g], ci[q]);
                        }
                        // Ad = Ad w + A (derivative in w), then A = A w + H, At = At w + H'
                        const cpx<double> wg = w[g];
                        Ad[g] = cadd(cmul(Ad[g], wg), A[g]);
                        A[g] = cadd(cmul(A[g], wg), cpx<double>{hr, hi});
                        At[g] = cadd(cmul(At[g], wg), cpx<double>{dr, di});
                    }
                }
#pragma unroll
                for (int g = 0; g < kGA; ++g) {
                    if (!live[g]) continue;
                    const int n = tn * kTN + wave * kGA + g;
                    // A_p = w dA/dw
                    const cpx<double> Ap = cmul(w[g], Ad[g]);
                    const cpx<double> Z = cmul(ph[g], A[g]);
                    // dZ/dr = -jk Z - (t/r) ph At ;  dZ/dalpha = j ph (Ap - P A)
                    const cpx<double> pAt = cmul(ph[g], At[g]);
                    const double f = t[g] * ir[g];
                    const cpx<double> Zr = {k * Z.im - f * pAt.re, -k * Z.re - f * pAt.im};
                    const cpx<double> q = cmul(ph[g], cpx<double>{Ap.re - P * A[g].re, Ap.im - P * A[g].im});
                    const cpx<double> Za = {-q.im, q.re};
                    const cpx<double> Zx = {ca[g] * Zr.re - sa[g] * ir[g] * Za.re,
                                            ca[g] * Zr.im - sa[g] * ir[g] * Za.im};
                    const cpx<double> Zy = {sa[g] * Zr.re + ca[g] * ir[g] * Za.re,
                                            sa[g] * Zr.im + ca[g] * ir[g] * Za.im};
                    const double2 v = a.W[size_t(n * nm + S) * a.ldw + size_t(m) * nm + T];
                    cx[g] += v.x * Zx.re - v.y * Zx.im;
                    cy[g] += v.x * Zy.re - v.y * Zy.im;
                }
            }
        }
    }

    // testing side: per lane over its 4 source antennas, then over the 4 waves
    __shared__ double red[4][kTM][2];
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int g = 0; g < kGA; ++g) {
        sx += cx[g];
        sy += cy[g];
    }
    red[wave][lane][0] = sx;
    red[wave][lane][1] = sy;
    __syncthreads();
    if (wave == 0 && m < a.n_ant) {
        double tx = 0.0, ty = 0.0;
        for (int q = 0; q < 4; ++q) {
            tx += red[q][lane][0];
            ty += red[q][lane][1];
        }
        a.part_m[(size_t(tn) * a.n_ant + m) * 2 + 0] = tx;
        a.part_m[(size_t(tn) * a.n_ant + m) * 2 + 1] = ty;
    }
    // source side: each (wave, g) sums over the 64 testing lanes
#pragma unroll
    for (int g = 0; g < kGA; ++g) {
        double vx = cx[g], vy = cy[g];
        for (int off = 32; off > 0; off >>= 1) {
            vx += __shfl_down(vx, off, 64);
            vy += __shfl_down(vy, off, 64);
        }
        const int n = tn * kTN + wave * kGA + g;
        if (lane == 0 && n < a.n_ant) {
            a.part_n[(size_t(tm) * a.n_ant + n) * 2 + 0] = vx;
            a.part_n[(size_t(tm) * a.n_ant + n) * 2 + 1] = vy;
        }
    }
}

// gx_i += sum_tn part_m - sum_tm part_n (fixed order)
__global__ void fill_vjp_sum_kernel(const double* __restrict__ part_m, const double* __restrict__ part_n, int n_ant,
                                    int tiles_m, int tiles_n, double* __restrict__ gx, double* __restrict__ gy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ant) return;
    double sx = 0.0, sy = 0.0;
    for (int q = 0; q < tiles_n; ++q) {
        sx += part_m[(size_t(q) * n_ant + i) * 2 + 0];
        sy += part_m[(size_t(q) * n_ant + i) * 2 + 1];
    }
    for (int q = 0; q < tiles_m; ++q) {
        sx -= part_n[(size_t(q) * n_ant + i) * 2 + 0];
        sy -= part_n[(size_t(q) * n_ant + i) * 2 + 1];
    }
    gx[i] += sx;
    gy[i] += sy;
}

__global__ void vjp_info_init(int32_t* info) {
    if (threadIdx.x == 0) info[0] = 0;
}

void vjp_tiles(int n_ant, int* tiles_m, int* tiles_n) {
    *tiles_m = (n_ant + kTM - 1) / kTM;
    *tiles_n = (n_ant + kTN - 1) / kTN;
}

// dst = op(src) for `batch` complex128 matrices (op: optional transpose and
// conjugate); rows x cols is the shape of src.
__global__ void __launch_bounds__(256)
    cmatrix_copy_kernel(int rows, int cols, const double2* __restrict__ src, int64_t lds, int64_t ss,
                        double2* __restrict__ dst, int64_t ldd, int64_t sd, int transpose, int conj) {
    const int b = blockIdx.z;
    __shared__ double2 tile[32][33];
    const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
    const double2* S = src + size_t(b) * ss;
    double2* D = dst + size_t(b) * sd;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int r = r0 + tx, c = c0 + j;
        double2 v = (r < rows && c < cols) ? S[size_t(c) * lds + r] : double2{0.0, 0.0};
        if (conj) v.y = -v.y;
        tile[j][tx] = v;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        if (transpose) {
            // dst (cols x rows): dst[r][c] at column r = r0 + j, row c = c0 + tx
            const int r = r0 + j, c = c0 + tx;
            if (r < rows && c < cols) D[size_t(r) * ldd + c] = tile[tx][j];
        } else {
            const int r = r0 + tx, c = c0 + j;
            if (r < rows && c < cols) D[size_t(c) * ldd + r] = tile[j][tx];
        }
    }
}

// gX[(i,T), q] = conj(w_T) gY[i, q]  (cotangent of X through Y = W^T X)
__global__ void __launch_bounds__(256)
    port_admittance_vjp_kernel(const char* __restrict__ models, int64_t model_stride, int n_mbf, int n_ant,
                               const double2* __restrict__ gY, int64_t ldy, int64_t sy, double2* __restrict__ gX,
                               int64_t ldx, int64_t sx) {
    const int f = blockIdx.y;
    const char* model = models + size_t(f) * model_stride;
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(model);
    const double2* w = reinterpret_cast<const double2*>(model + h->off_port);
    const int64_t n = int64_t(n_ant) * n_mbf, total = n * n_ant;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t q = e / n, row = e % n;
        const int64_t i = row / n_mbf, T = row % n_mbf;
        const double2 g = gY[size_t(f) * sy + q * ldy + i];
        const double2 ww = w[T];
        gX[size_t(f) * sx + q * ldx + row] = double2{ww.x * g.x + ww.y * g.y, ww.x * g.y - ww.y * g.x};
    }
}

}  // namespace
}  // namespace harp

using namespace harp;

extern "C" harp_status harp_fill_vjp_ws(int32_t n_ant, size_t* bytes) {
    if (!bytes || n_ant <= 0) return HARP_E_ARG;
    int tm, tn;
    vjp_tiles(n_ant, &tm, &tn);
    *bytes = size_t(align256(int64_t(tn) * n_ant * 16) + align256(int64_t(tm) * n_ant * 16));
    return HARP_OK;
}

extern "C" harp_status harp_fill_vjp(const void* d_model, int32_t n_mbf, int32_t Q, const double* d_x,
                                     const double* d_y, int32_t n_ant, double ri, const void* d_W, int64_t ldw,
                                     double* d_gx, double* d_gy, int32_t* d_info, void* d_ws, size_t ws_bytes,
                                     hipStream_t stream) {
    if (!d_model || !d_x || !d_y || !d_W || !d_gx || !d_gy || !d_info || n_mbf <= 0 || n_ant <= 0) return HARP_E_ARG;
    if (Q < 2 || Q > 8 || ldw < int64_t(n_ant) * n_mbf) return HARP_E_ARG;
    size_t need;
    harp_fill_vjp_ws(n_ant, &need);
    if (!d_ws || ws_bytes < need) return HARP_E_WORKSPACE;
    int tm, tn;
    vjp_tiles(n_ant, &tm, &tn);
    VjpArgs a;
    a.model = static_cast<const char*>(d_model);
    a.x = d_x;
    a.y = d_y;
    a.n_ant = n_ant;
    a.n_mbf = n_mbf;
    a.ri = ri;
    a.W = static_cast<const double2*>(d_W);
    a.ldw = ldw;
    a.part_m = static_cast<double*>(d_ws);
    a.part_n = reinterpret_cast<double*>(static_cast<char*>(d_ws) + align256(int64_t(tn) * n_ant * 16));
    a.info = d_info;
    // the FP64 coefficient table sits right after the 256-byte header
    const double* coef = reinterpret_cast<const double*>(a.model + 256);
    const dim3 grid(unsigned(tm * tn));
    hipLaunchKernelGGL(vjp_info_init, dim3(1), dim3(64), 0, stream, d_info);
    HARP_LAUNCH_CHECK();
    switch (Q) {
#define HARP_VJP_CASE(QQ)                                                                             \
    case QQ:                                                                                          \
        HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,                                                \
                         hipLaunchKernelGGL((fill_vjp_kernel<QQ>), grid, dim3(256), 0, stream, a, coef)); \
        break;
        HARP_VJP_CASE(2)
        HARP_VJP_CASE(3)
        HARP_VJP_CASE(4)
        HARP_VJP_CASE(5)
        HARP_VJP_CASE(6)
        HARP_VJP_CASE(7)
        HARP_VJP_CASE(8)
#undef HARP_VJP_CASE
    }
    HARP_LAUNCH_CHECK();
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(fill_vjp_sum_kernel, dim3((n_ant + 255) / 256), dim3(256), 0, stream,
                                        a.part_m, a.part_n, n_ant, tm, tn, d_gx, d_gy));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

extern "C" harp_status harp_cmatrix_copy(int32_t rows, int32_t cols, int32_t batch, const void* d_src, int64_t lds,
                                         int64_t stride_src, void* d_dst, int64_t ldd, int64_t stride_dst,
                                         int32_t transpose, int32_t conj, hipStream_t stream) {
    if (rows < 0 || cols < 0 || batch < 0 || (rows * int64_t(cols) > 0 && (!d_src || !d_dst))) return HARP_E_ARG;
    if (rows == 0 || cols == 0 || batch == 0) return HARP_OK;
    if (lds < rows || ldd < (transpose ? cols : rows) || batch > 65535) return HARP_E_ARG;
    if (d_src == d_dst && transpose) return HARP_E_ARG;
    const dim3 grid(unsigned((rows + 31) / 32), unsigned((cols + 31) / 32), unsigned(batch));
    if (grid.y > 65535) return HARP_E_ARG;
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(cmatrix_copy_kernel, grid, dim3(256), 0, stream, rows, cols,
                                        static_cast<const double2*>(d_src), lds, stride_src,
                                        static_cast<double2*>(d_dst), ldd, stride_dst, transpose, conj));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

extern "C" harp_status harp_port_admittance_vjp(const void* d_models, int64_t model_stride, int32_t n_freq,
                                                int32_t n_mbf, int32_t n_ant, const void* d_gY, int64_t ldy,
                                                int64_t stride_y, void* d_gX, int64_t ldx, int64_t stride_x,
                                                hipStream_t stream) {
    if (!d_models || !d_gY || !d_gX || n_freq <= 0 || n_mbf <= 0 || n_ant <= 0) return HARP_E_ARG;
    if (ldy < n_ant || ldx < int64_t(n_ant) * n_mbf || n_freq > 65535) return HARP_E_ARG;
    const int64_t total = int64_t(n_ant) * n_mbf * n_ant;
    const unsigned blocks = unsigned(std::min<int64_t>((total + 255) / 256, 4096));
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(port_admittance_vjp_kernel, dim3(blocks, unsigned(n_freq)), dim3(256), 0,
                                        stream, static_cast<const char*>(d_models), model_stride, n_mbf, n_ant,
                                        static_cast<const double2*>(d_gY), ldy, stride_y,
                                        static_cast<double2*>(d_gX), ldx, stride_x));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}
