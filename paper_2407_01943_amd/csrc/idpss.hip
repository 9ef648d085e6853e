// Interpolated-DPSS tapers (Table 3 step 3, the branch for a nominal band
// centred at 0; Table 3 in Sec. 3.7, approximating the GPSS tapers by DPSS):
//   (a) the DPSS of length N and half-bandwidth f_w D on the uniform grid
//       u_m = t_1 + m D, D = (t_N - t_1) / (N - 1): the GPSS tapers of the
//       integer lattice 0..N-1 with f_max = 1/2 (R(B) = I), computed by the
//       lattice GEP path;
//   (b) the natural cubic spline through (u_m, v_m), evaluated at t_n;
//   (c) the scale that makes w^T R(B) w = 2 f_w (Eq. of the normalisation
//       requirement), and the sign reading of the GEP tapers.
//
// Spline second derivatives.  In grid units the natural spline's second
// derivatives solve M_{i-1} + 4 M_i + M_{i+1} = r_i = 6 (v_{i+1} - 2 v_i +
// v_{i-1}) for 0 < i < N-1 with M_0 = M_{N-1} = 0.  Extending r oddly about
// both ends (period 2 (N - 1)) turns this into the bi-infinite Toeplitz
// system, whose inverse is g_k = z^|k| / (2 sqrt 3), z = sqrt 3 - 2: the odd
// extension of the solution vanishes at the ends, so the convolution with g
// solves the finite system exactly.  |z|^31 < 2e-18, so 30 taps on each side
// leave an error below 1e-17 of max |r|; every M_i is an independent sum.
#include <cmath>

#include "m2n_common.hpp"

namespace m2n {

namespace {

constexpr int IT = 256;        // threads per workgroup
constexpr int SPL_L = 30;      // spline filter taps on each side
constexpr int ID_KMAX = 32;    // tapers per call
constexpr int QT = 128;        // columns of a quadratic-form tile

// flags: bit 0 a non-finite t_n, bit 1 t_n <= t_{n-1}, bit 2 a t_n that is
// not an integer of magnitude <= 4e15
__global__ __launch_bounds__(IT) void k_id_check(const double* __restrict__ t, int64_t N,
                                                 unsigned* __restrict__ flags) {
    const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
    unsigned f = 0;
    if (n < N) {
        const double v = t[n];
        if (!std::isfinite(v)) f |= 1u;
        if (n > 0 && !(v > t[n - 1])) f |= 2u;
        if (!(v == rint(v)) || !(fabs(v) <= 4e15)) f |= 4u;
    }
    if (f) atomicOr(flags, f);
}

__global__ __launch_bounds__(IT) void k_id_grid(double* __restrict__ u, int64_t N) {
    const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (n < N) u[n] = (double)n;
}

// r~_j of taper row v (odd extension of r about 0 and N - 1)
__device__ __forceinline__ double r_ext(const double* __restrict__ v, int64_t N, int64_t j) {
    if (j > 0 && j < N - 1) return 6.0 * ((v[j + 1] - 2.0 * v[j]) + v[j - 1]);
    const int64_t P = 2 * (N - 1);
    int64_t jj = j % P;
    if (jj < 0) jj += P;
    double sg = 1.0;
    if (jj > N - 1) {
        jj = P - jj;
        sg = -1.0;
    }
    if (jj == 0 || jj == N - 1) return 0.0;
    return sg * 6.0 * ((v[jj + 1] - 2.0 * v[jj]) + v[jj - 1]);
}

// M[k N + i] = sum_{|d| <= SPL_L} g_d r~_{i+d}; blockIdx.y = taper.  The
// workgroup's IT + 2 SPL_L right-hand sides are formed once into LDS.
__global__ __launch_bounds__(IT) void k_id_spline(const double* __restrict__ v, int64_t N,
                                                  double* __restrict__ M) {
    __shared__ double rs[IT + 2 * SPL_L];
    const int64_t i0 = (int64_t)blockIdx.x * IT;
    const double* __restrict__ vk = v + (int64_t)blockIdx.y * N;
    for (int e = threadIdx.x; e < IT + 2 * SPL_L; e += IT) rs[e] = N >= 3 ? r_ext(vk, N, i0 - SPL_L + e) : 0.0;
    __syncthreads();
    const int64_t i = i0 + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    if (N >= 3 && i > 0 && i < N - 1) {
        const double z = sqrt(3.0) - 2.0;
        const int c = threadIdx.x + SPL_L;
        double zp = 1.0;
        acc = rs[c];
        for (int d = 1; d <= SPL_L; ++d) {
            zp *= z;
            acc += zp * (rs[c - d] + rs[c + d]);
        }
        acc *= 1.0 / (2.0 * sqrt(3.0));
    }
    M[(int64_t)blockIdx.y * N + i] = acc;
}

// w[k N + n] = S_k(t_n), the natural spline of taper k in grid units:
// x = (t_n - t_1) / D, m = floor(x) in [0, N - 2], s = x - m,
// S = (1-s) v_m + s v_{m+1} + ((1-s)^3 - (1-s)) M_m / 6 + (s^3 - s) M_{m+1} / 6
__global__ __launch_bounds__(IT) void k_id_eval(const double* __restrict__ t, int64_t N, double t0, double D,
                                                const double* __restrict__ v, const double* __restrict__ M,
                                                int K, double* __restrict__ w) {
    const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (n >= N) return;
    const double x = (t[n] - t0) / D;
    int64_t m = (int64_t)floor(x);
    m = m < 0 ? 0 : (m > N - 2 ? N - 2 : m);
    const double s = x - (double)m, a = 1.0 - s;
    const double ca = (a * a * a - a) * (1.0 / 6.0), cs = (s * s * s - s) * (1.0 / 6.0);
    for (int k = 0; k < K; ++k) {
        const int64_t o = (int64_t)k * N + m;
        w[(int64_t)k * N + n] = (a * v[o] + s * v[o + 1]) + (ca * M[o] + cs * M[o + 1]);
    }
}

__device__ __forceinline__ double id_block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < IT / 64; ++q) s += red[q];
    return s;
}

// per workgroup, per taper: sum w^2, sum w, sum (tbar - t) w / span
__global__ __launch_bounds__(IT) void k_id_sums(const double* __restrict__ t, int64_t N, int K,
                                                const double* __restrict__ w, double* __restrict__ part) {
    __shared__ double red[IT / 64];
    const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
    const double tbar = 0.5 * (t[0] + t[N - 1]);
    const double span = N > 1 ? t[N - 1] - t[0] : 1.0;
    const double lev = n < N ? (tbar - t[n]) / span : 0.0;
    for (int k = 0; k < K; ++k) {
        const double x = n < N ? w[(int64_t)k * N + n] : 0.0;
        const double a = id_block_sum(x * x, red);
        const double b = id_block_sum(x, red);
        const double c = id_block_sum(lev * x, red);
        if (threadIdx.x == 0) {
            part[((int64_t)blockIdx.x * K + k) * 3 + 0] = a;
            part[((int64_t)blockIdx.x * K + k) * 3 + 1] = b;
            part[((int64_t)blockIdx.x * K + k) * 3 + 2] = c;
        }
    }
}

// sin(2 pi f tau) / (pi tau) with the argument reduced exactly first
__device__ __forceinline__ double id_sinc(double f, double tau) {
    if (tau == 0.0) return 2.0 * f;
    const double u = 2.0 * f * tau;
    double r = u - 2.0 * rint(0.5 * u);
    if (r > 0.5) r = 1.0 - r;
    else if (r < -0.5) r = -1.0 - r;
    return sinpi(r) / (M_PI * tau);
}

// partial quadratic forms w_k^T R(B) w_k: workgroup (bx, by, bz) takes rows
// n in [bx IT, (bx + 1) IT) against columns m in chunk by of cm columns for
// the tapers k in [QK bz, QK bz + QK), staged through LDS QT columns at a
// time.  R(B) is symmetric, so only m >= n is summed, off-diagonal pairs
// twice: acc_k(n) = w_k(n) R(B)_nn + 2 sum_{m > n} w_k(m) R(B)_{nm}; tiles
// wholly below the workgroup's rows are skipped.  The workgroup then sums
// w_k(n) acc_k(n) into part[(by gx + bx) K + k]
constexpr int QK = 8;
__global__ __launch_bounds__(IT) void k_id_quad(const double* __restrict__ t, int64_t N, int K, double fmax,
                                                const double* __restrict__ w, int64_t cm,
                                                double* __restrict__ part) {
    __shared__ double ts[QT];
    __shared__ double ws[QK][QT];
    __shared__ double red[IT / 64];
    const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
    const double tn = n < N ? t[n] : 0.0;
    const int k0 = QK * (int)blockIdx.z;
    const int kn = K - k0 < QK ? K - k0 : QK;
    double acc[QK];
#pragma unroll
    for (int k = 0; k < QK; ++k) acc[k] = 0.0;
    const int64_t m0 = (int64_t)blockIdx.y * cm;
    const int64_t m1 = m0 + cm < N ? m0 + cm : N;
    const int64_t rlo = (int64_t)blockIdx.x * IT;   // first row of the workgroup
    for (int64_t mb = m0; mb < m1; mb += QT) {
        const int cnt = (int)(m1 - mb < QT ? m1 - mb : QT);
        if (mb + cnt <= rlo) continue;   // every m < every n of this workgroup (uniform)
        __syncthreads();
        for (int e = threadIdx.x; e < QT; e += IT) ts[e] = e < cnt ? t[mb + e] : 0.0;
        for (int e = threadIdx.x; e < QK * QT; e += IT) {
            const int k = e / QT, j = e % QT;
            ws[k][j] = (j < cnt && k < kn) ? w[(int64_t)(k0 + k) * N + mb + j] : 0.0;
        }
        __syncthreads();
        if (n < N)
            for (int j = 0; j < cnt; ++j) {
                const int64_t m = mb + j;
                if (m < n) continue;
                const double s = (m == n ? 1.0 : 2.0) * id_sinc(fmax, tn - ts[j]);
#pragma unroll
                for (int k = 0; k < QK; ++k) acc[k] += ws[k][j] * s;
            }
    }
#pragma unroll
    for (int k = 0; k < QK; ++k) {
        const double x = (n < N && k < kn) ? w[(int64_t)(k0 + k) * N + n] * acc[k] : 0.0;
        const double q = id_block_sum(x, red);
        if (threadIdx.x == 0 && k < kn) part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * K + k0 + k] = q;
    }
}

// scale and sign of taper k = blockIdx.x (one wavefront): the lanes sum
// interleaved partials, then a butterfly (a fixed order); q_k is
// 2 f_max sum w^2 on a lattice, else the quadratic form
__global__ __launch_bounds__(64) void k_id_scale(int K, double fw, double fmax, const double* __restrict__ sums,
                                                 int nsum, const double* __restrict__ quad, int nquad,
                                                 double* __restrict__ sc) {
    const int k = blockIdx.x, l = threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0, q = 0.0;
    for (int g = l; g < nsum; g += 64) {
        a += sums[((int64_t)g * K + k) * 3 + 0];
        b += sums[((int64_t)g * K + k) * 3 + 1];
        c += sums[((int64_t)g * K + k) * 3 + 2];
    }
    if (quad)
        for (int g = l; g < nquad; g += 64) q += quad[(int64_t)g * K + k];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
        q += __shfl_xor(q, o, 64);
    }
    if (l == 0) {
        if (!quad) q = 2.0 * fmax * a;
        const double key = fabs(b) >= fabs(c) ? b : c;
        const double s = q > 0.0 ? sqrt(2.0 * fw / q) : 0.0;
        sc[k] = key < 0.0 ? -s : s;
    }
}

__global__ __launch_bounds__(IT) void k_id_apply(double* __restrict__ w, int64_t N, int K,
                                                 const double* __restrict__ sc) {
    const int64_t n = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (n >= N) return;
    for (int k = 0; k < K; ++k) w[(int64_t)k * N + n] *= sc[k];
}

}  // namespace

int idpss_run(Ctx* ctx, hipStream_t st, const double* t, int64_t N, double fmax, double fw, int K,
              double* w, double* lambda) {
    if (N < 2 || K < 1 || K > ID_KMAX || K > N) {
        set_error("need N >= 2 and 1 <= K <= min(N, %d) (N = %lld, K = %d)", ID_KMAX, (long long)N, K);
        return M2N_ERR_ARG;
    }
    if (!std::isfinite(fmax) || !std::isfinite(fw) || !(fw > 0.0) || !(fw < fmax)) {
        set_error("need 0 < fw < fmax (fw = %g, fmax = %g)", fw, fmax);
        return M2N_ERR_ARG;
    }
    const int nb = (int)((N + IT - 1) / IT);
    void *vfl, *vu, *vv, *vM, *vs;
    M2N_TRY(ctx->workspace("id_flags", 64, &vfl));
    M2N_TRY(ctx->workspace("id_u", sizeof(double) * (size_t)N, &vu));
    M2N_TRY(ctx->workspace("id_v", sizeof(double) * (size_t)K * N, &vv));
    M2N_TRY(ctx->workspace("id_M", sizeof(double) * (size_t)K * N, &vM));
    M2N_TRY(ctx->workspace("id_sums", sizeof(double) * (size_t)nb * K * 3, &vs));
    void* vsc;
    M2N_TRY(ctx->workspace("id_scale", sizeof(double) * ID_KMAX, &vsc));
    unsigned* flags = (unsigned*)vfl;
    M2N_HIP(hipMemsetAsync(flags, 0, 64, st));
    {
        M2N_PROF(ctx, st, "k_id_check");
        hipLaunchKernelGGL(k_id_check, dim3((unsigned)nb), dim3(IT), 0, st, t, N, flags);
    }
    M2N_HIP(hipGetLastError());
    unsigned hf = 0;
    double ends[2] = {0.0, 0.0};
    M2N_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    M2N_HIP(hipMemcpyAsync(&ends[0], t, sizeof(double), hipMemcpyDeviceToHost, st));
    M2N_HIP(hipMemcpyAsync(&ends[1], t + (N - 1), sizeof(double), hipMemcpyDeviceToHost, st));
    M2N_HIP(hipStreamSynchronize(st));
    if (hf & 1u) {
        set_error("non-finite sampling time");
        return M2N_ERR_ARG;
    }
    if (hf & 2u) {
        set_error("sampling times not strictly increasing");
        return M2N_ERR_T_ORDER;
    }
    const double t0 = ends[0], D = (ends[1] - ends[0]) / (double)(N - 1);
    const double Wn = fw * D;   // half-bandwidth in cycles per grid step
    if (!(Wn < 0.5)) {
        set_error("f_w (t_N - t_1) / (N - 1) = %g must be below 1/2", Wn);
        return M2N_ERR_ARG;
    }
    double* u = (double*)vu;
    double* v = (double*)vv;
    double* M = (double*)vM;
    {
        M2N_PROF(ctx, st, "k_id_grid");
        hipLaunchKernelGGL(k_id_grid, dim3((unsigned)nb), dim3(IT), 0, st, u, N);
    }
    M2N_HIP(hipGetLastError());
    // (a) DPSS = GPSS tapers of the unit lattice with f_max = 1/2
    M2N_TRY(gep_run(ctx, st, u, N, 0.5, Wn, K, v, lambda));
    // (b) spline
    {
        M2N_PROF(ctx, st, "k_id_spline");
        hipLaunchKernelGGL(k_id_spline, dim3((unsigned)nb, (unsigned)K), dim3(IT), 0, st, (const double*)v, N, M);
    }
    {
        M2N_PROF(ctx, st, "k_id_eval");
        hipLaunchKernelGGL(k_id_eval, dim3((unsigned)nb), dim3(IT), 0, st, t, N, t0, D, (const double*)v,
                           (const double*)M, K, w);
    }
    M2N_HIP(hipGetLastError());
    // (c) scale and sign
    {
        M2N_PROF(ctx, st, "k_id_sums");
        hipLaunchKernelGGL(k_id_sums, dim3((unsigned)nb), dim3(IT), 0, st, t, N, K, (const double*)w,
                           (double*)vs);
    }
    const double tf = 2.0 * fmax;
    const bool lattice = !(hf & 4u) && tf == std::rint(tf) && tf >= 1.0;
    const double* quad = nullptr;
    int nquad = 0;
    if (!lattice) {
        const int64_t cm = 1024;
        const int nc = (int)((N + cm - 1) / cm);
        void* vq;
        M2N_TRY(ctx->workspace("id_quad", sizeof(double) * (size_t)nb * nc * K, &vq));
        {
            M2N_PROF(ctx, st, "k_id_quad");
            hipLaunchKernelGGL(k_id_quad, dim3((unsigned)nb, (unsigned)nc, (unsigned)((K + QK - 1) / QK)),
                               dim3(IT), 0, st, t, N, K, fmax,
                               (const double*)w, cm, (double*)vq);
        }
        quad = (const double*)vq;
        nquad = nb * nc;
    }
    {
        M2N_PROF(ctx, st, "k_id_scale");
        hipLaunchKernelGGL(k_id_scale, dim3((unsigned)K), dim3(64), 0, st, K, fw, fmax, (const double*)vs, nb,
                           quad, nquad, (double*)vsc);
    }
    {
        M2N_PROF(ctx, st, "k_id_apply");
        hipLaunchKernelGGL(k_id_apply, dim3((unsigned)nb), dim3(IT), 0, st, w, N, K, (const double*)vsc);
    }
    M2N_HIP(hipGetLastError());
    return M2N_OK;
}

}  // namespace m2n
