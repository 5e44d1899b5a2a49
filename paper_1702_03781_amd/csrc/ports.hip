// Port excitation and port admittances (Sections I and II-C).
//
// One port per element drives its MBFs with the weights w_T stored in the
// model; a unit voltage at port j gives the right-hand side column
// B[:, j] = e_j (x) w, and the current at port i of solution column j is
// Y_ij = sum_T w_T X[i N_m + T, j]  (Y = W^T X).
#include "common.hpp"
#include "prof.hpp"

namespace harp {
namespace {

// The system behind matrix f: its model, antenna count and port count (all
// n_ant antennas, model f and n_cols ports without descriptors).  False for a
// descriptor out of range: its matrices are then written as zeros.
__device__ inline bool system_of(const harp_system* sys, int n_models, int f, int n_ant, int n_cols, int* model,
                                 int* ns, int* np) {
    *model = f;
    *ns = n_ant;
    *np = n_cols;
    if (!sys) return true;
    const harp_system d = sys[f];
    const int ports = d.n_ports == 0 ? d.n_ant : d.n_ports;
    if (d.model < 0 || d.model >= n_models || d.n_ant < 1 || d.n_ant > n_ant || ports < 0 || ports > d.n_ant ||
        ports > n_cols)
        return false;
    *model = d.model;
    *ns = d.n_ant;
    *np = ports;
    return true;
}

// B (complex128, n x n_cols per matrix, n = n_ant n_mbf): one thread per
// entry; column j < ports is e_j (x) w, the rest (and the rows of padding
// antennas) zero.
__global__ void __launch_bounds__(256)
    port_rhs_kernel(const char* __restrict__ models, int64_t model_stride, int n_mbf, int n_ant, int n_cols,
                    double2* __restrict__ B, int64_t ldb, int64_t stride_b, const harp_system* __restrict__ sys,
                    int n_models) {
    const int f = blockIdx.y;
    int mi, ns, np;
    const bool ok = system_of(sys, n_models, f, n_ant, n_cols, &mi, &ns, &np);
    const char* model = models + size_t(ok ? mi : 0) * model_stride;
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(model);
    const double2* w = reinterpret_cast<const double2*>(model + h->off_port);
    const int64_t n = int64_t(n_ant) * n_mbf;
    const int64_t total = n * n_cols;
    double2* Bf = B + size_t(f) * stride_b;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t col = e / n, row = e % n;
        const int64_t ant = row / n_mbf, T = row % n_mbf;
        double2 v = {0.0, 0.0};
        if (ok && ant == col && col < np) v = w[T];
        Bf[col * ldb + row] = v;
    }
}

// Y (complex128, n_ant x n_cols per matrix): Y_ij = sum_T w_T X[i N_m + T, j]
// for antennas i < ns and ports j < np, zero elsewhere.  A wave reads 64
// consecutive rows of one column of X (N_m lanes per antenna, 64 / N_m
// antennas), forms w_T x in each lane and sums the N_m lanes of an antenna
// through LDS: contiguous loads instead of one 16-byte piece per antenna row.
__global__ void __launch_bounds__(256)
    port_admittance_kernel(const char* __restrict__ models, int64_t model_stride, int n_mbf, int n_ant, int n_cols,
                           const double2* __restrict__ X, int64_t ldx, int64_t stride_x, double2* __restrict__ Y,
                           int64_t ldy, int64_t stride_y, const harp_system* __restrict__ sys, int n_models) {
    const int f = blockIdx.y;
    int mi, ns, np;
    const bool ok = system_of(sys, n_models, f, n_ant, n_cols, &mi, &ns, &np);
    const char* model = models + size_t(ok ? mi : 0) * model_stride;
    const ModelHeader* h = reinterpret_cast<const ModelHeader*>(model);
    const double2* w = reinterpret_cast<const double2*>(model + h->off_port);
    const double2* Xf = X + size_t(f) * stride_x;
    double2* Yf = Y + size_t(f) * stride_y;
    __shared__ double2 part[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = 64 / n_mbf;                     // antennas per wave segment
    const int ai = lane / n_mbf, T = lane % n_mbf;
    const int64_t segs = (int64_t(n_ant) + per - 1) / per;
    const int64_t total = segs * n_cols;            // (segment, column) units, one per wave
    const double2 wt = w[T < n_mbf ? T : 0];
    for (int64_t u0 = int64_t(blockIdx.x) * 4; u0 < total; u0 += int64_t(gridDim.x) * 4) {
        const int64_t u = u0 + wave;
        const bool unit = u < total;
        const int64_t j = unit ? u / segs : 0;
        const int64_t i = unit ? (u % segs) * per + ai : 0;
        double2 v = {0.0, 0.0};
        if (unit && ok && ai < per && i < ns && j < np) {
            const double2 x = Xf[j * ldx + i * n_mbf + T];
            v.x = wt.x * x.x - wt.y * x.y;
            v.y = wt.x * x.y + wt.y * x.x;
        }
        part[wave][lane] = v;
        __syncthreads();
        if (unit && T == 0 && ai < per && i < n_ant) {
            double re = 0.0, im = 0.0;
            for (int t = 0; t < n_mbf; ++t) {
                re += part[wave][lane + t].x;
                im += part[wave][lane + t].y;
            }
            Yf[j * ldy + i] = double2{re, im};
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace harp

using namespace harp;

namespace {

harp_status rhs_launch(const void* d_models, int64_t model_stride, int32_t n_mat, int32_t n_mbf, int32_t n_ant,
                       int32_t n_cols, void* d_B, int64_t ldb, int64_t stride_b, const harp_system* d_sys,
                       int32_t n_models, hipStream_t stream) {
    if (!d_models || !d_B || n_mat <= 0 || n_mat > 65535 || n_mbf <= 0 || n_ant <= 0 || n_cols <= 0)
        return HARP_E_ARG;
    const int64_t n = int64_t(n_ant) * n_mbf;
    if (ldb < n || (n_mat > 1 && stride_b < ldb * n_cols)) return HARP_E_ARG;
    const int64_t total = n * n_cols;
    const unsigned blocks = unsigned(std::min<int64_t>((total + 255) / 256, 4096));
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(port_rhs_kernel, dim3(blocks, unsigned(n_mat)), dim3(256), 0, stream,
                                        static_cast<const char*>(d_models), model_stride, n_mbf, n_ant, n_cols,
                                        static_cast<double2*>(d_B), ldb, stride_b, d_sys, n_models));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

harp_status admittance_launch(const void* d_models, int64_t model_stride, int32_t n_mat, int32_t n_mbf,
                              int32_t n_ant, int32_t n_cols, const void* d_X, int64_t ldx, int64_t stride_x,
                              void* d_Y, int64_t ldy, int64_t stride_y, const harp_system* d_sys, int32_t n_models,
                              hipStream_t stream) {
    if (!d_models || !d_X || !d_Y || n_mat <= 0 || n_mat > 65535 || n_mbf <= 0 || n_ant <= 0 || n_cols <= 0)
        return HARP_E_ARG;
    const int64_t n = int64_t(n_ant) * n_mbf;
    if (ldx < n || ldy < n_ant) return HARP_E_ARG;
    if (n_mat > 1 && (stride_x < ldx * n_cols || stride_y < ldy * n_cols)) return HARP_E_ARG;
    if (n_mbf > 64) return HARP_E_ARG;
    const int per = 64 / n_mbf;
    const int64_t units = ((int64_t(n_ant) + per - 1) / per) * n_cols;
    const unsigned blocks = unsigned(std::min<int64_t>((units + 3) / 4, 4096));
    HARP_PROF_LAUNCH(HARP_K_AUX, stream, 0.0, 0.0,
                     hipLaunchKernelGGL(port_admittance_kernel, dim3(blocks, unsigned(n_mat)), dim3(256), 0,
                                        stream, static_cast<const char*>(d_models), model_stride, n_mbf, n_ant, n_cols,
                                        static_cast<const double2*>(d_X), ldx, stride_x, static_cast<double2*>(d_Y),
                                        ldy, stride_y, d_sys, n_models));
    HARP_LAUNCH_CHECK();
    return HARP_OK;
}

}  // namespace

extern "C" harp_status harp_port_rhs(const void* d_models, int64_t model_stride, int32_t n_freq, int32_t n_mbf,
                                     int32_t n_ant, void* d_B, int64_t ldb, int64_t stride_b,
                                     hipStream_t stream) {
    return rhs_launch(d_models, model_stride, n_freq, n_mbf, n_ant, n_ant, d_B, ldb, stride_b, nullptr, 0, stream);
}

extern "C" harp_status harp_port_admittance(const void* d_models, int64_t model_stride, int32_t n_freq,
                                            int32_t n_mbf, int32_t n_ant, const void* d_X, int64_t ldx,
                                            int64_t stride_x, void* d_Y, int64_t ldy, int64_t stride_y,
                                            hipStream_t stream) {
    return admittance_launch(d_models, model_stride, n_freq, n_mbf, n_ant, n_ant, d_X, ldx, stride_x, d_Y, ldy,
                             stride_y, nullptr, 0, stream);
}

extern "C" harp_status harp_port_rhs_systems(const void* d_models, int64_t model_stride, int32_t n_models,
                                             int32_t n_mbf, const harp_system* d_sys, int32_t n_sys,
                                             int32_t n_ant_pad, int32_t n_ports_pad, void* d_B, int64_t ldb,
                                             int64_t stride_b, hipStream_t stream) {
    if (!d_sys || n_models <= 0) return HARP_E_ARG;
    return rhs_launch(d_models, model_stride, n_sys, n_mbf, n_ant_pad, n_ports_pad, d_B, ldb, stride_b, d_sys,
                      n_models, stream);
}

extern "C" harp_status harp_port_admittance_systems(const void* d_models, int64_t model_stride, int32_t n_models,
                                                    int32_t n_mbf, const harp_system* d_sys, int32_t n_sys,
                                                    int32_t n_ant_pad, int32_t n_ports_pad, const void* d_X,
                                                    int64_t ldx, int64_t stride_x, void* d_Y, int64_t ldy,
                                                    int64_t stride_y, hipStream_t stream) {
    if (!d_sys || n_models <= 0) return HARP_E_ARG;
    return admittance_launch(d_models, model_stride, n_sys, n_mbf, n_ant_pad, n_ports_pad, d_X, ldx, stride_x, d_Y,
                             ldy, stride_y, d_sys, n_models, stream);
}
