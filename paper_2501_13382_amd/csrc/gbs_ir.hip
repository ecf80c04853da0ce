// Broadband synthesis on the device: the beam sum's spectrum at a grid of
// frequencies turned into a time signal per receiver (the time-domain form
// of Eq. (1); the paper steps its field in time, Table 2).  With the
// exp(-i omega t) convention the real pressure is
//   h[m] = 2 df Re sum_n w_n P_n exp(-2 pi i f_n m dt),  f_n = (bin0 + n) df,  dt = 1 / (n_fft df),
// which is the real part of a length-n_fft DFT of the windowed, zero-padded
// spectrum.  One workgroup transforms one (source, receiver) row in LDS:
// bit-reversed load, then log2(n_fft) radix-2 butterfly stages in place.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace gbs {

// tw[k] = exp(-2 pi i k / n), k < n / 2.
__global__ void k_ir_twiddles(int n, double2* __restrict__ tw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n / 2) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)n, &s, &c);
    tw[k] = make_double2(c, -s);
}

// spec[(src * n_rcv + r) * n_fft + bin_off + b] = w[b0 + b] * P[src][b][r] for
// the nb bins of one forward call (P job-major: job = src * nb + b).
__global__ void k_ir_scatter(const double* __restrict__ P, int n_src, int nb, int64_t n_rcv, int bin_off,
                             const double* __restrict__ window, int b0, int n_fft, double2* __restrict__ spec) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)n_src * nb * n_rcv;
    if (t >= n) return;
    const int b = (int)(t % nb);                        // bins fastest: neighbouring threads write neighbours
    const int64_t sr = t / nb;
    const int src = (int)(sr / n_rcv);
    const int64_t r = sr - (int64_t)src * n_rcv;
    const double w = window ? window[b0 + b] : 1.0;
    const double* p = P + 2 * (((int64_t)src * nb + b) * n_rcv + r);
    spec[sr * n_fft + bin_off + b] = make_double2(w * p[0], w * p[1]);
}

// h[row][m] = scale * Re(DFT(spec[row]))[m], m < n_t; dynamic LDS of n_fft double2.
__global__ __launch_bounds__(256) void k_ir_fft(const double2* __restrict__ spec, int n_fft, int log2n,
                                                const double2* __restrict__ tw, double scale, int n_t,
                                                double* __restrict__ h) {
    extern __shared__ double2 x[];
    const int64_t row = blockIdx.x;
    const double2* in = spec + row * n_fft;
    for (int i = threadIdx.x; i < n_fft; i += blockDim.x) x[i] = in[__brev((unsigned)i) >> (32 - log2n)];
    __syncthreads();
    for (int s = 1; s <= log2n; ++s) {
        const int half = 1 << (s - 1);
        for (int j = threadIdx.x; j < n_fft / 2; j += blockDim.x) {
            const int pos = j & (half - 1);
            const int i0 = ((j >> (s - 1)) << s) + pos, i1 = i0 + half;
            const double2 w = tw[pos << (log2n - s)];
            const double2 b = x[i1];
            const double2 t = make_double2(w.x * b.x - w.y * b.y, w.x * b.y + w.y * b.x);
            const double2 a = x[i0];
            x[i0] = make_double2(a.x + t.x, a.y + t.y);
            x[i1] = make_double2(a.x - t.x, a.y - t.y);
        }
        __syncthreads();
    }
    double* out = h + row * n_t;
    for (int m = threadIdx.x; m < n_t; m += blockDim.x) out[m] = scale * x[m].x;
}

}  // namespace gbs
