// Type-independent FP64 kernels: fixed-order reduction of partial sums, the
// norm / breakdown decision of one Gram-Schmidt step, and the energy sum.
#include <algorithm>

#include "mar_device.h"
#include "mar_internal.h"

namespace mar {

// out[o] = sum_c part[c * L + o] for o < L, summed in a fixed order (chunk
// lanes strided by CL, then the CL lane sums in order). When h != nullptr the
// first nk*B outputs are also the subspace-matrix column n: o = k * B + b is
// written to h[b][k][n].
template <int OPW>
__global__ __launch_bounds__(WG) void k_reduce(const double* __restrict__ part, int64_t nchunks, int64_t L,
                                               double* __restrict__ out, double* __restrict__ h, int B, int nu,
                                               int n, int64_t hL) {
    constexpr int CL = WG / OPW;  // chunk lanes
    const int oi = threadIdx.x % OPW, cl = threadIdx.x / OPW;
    const int64_t o = (int64_t)blockIdx.x * OPW + oi;
    double s0 = 0.0, s1 = 0.0;
    if (o < L) {
        int64_t c = cl;
        for (; c + CL < nchunks; c += 2 * CL) {
            s0 += part[c * L + o];
            s1 += part[(c + CL) * L + o];
        }
        if (c < nchunks) s0 += part[c * L + o];
    }
    __shared__ double lds[WG];
    lds[threadIdx.x] = s0 + s1;
    __syncthreads();
    if (cl == 0 && o < L) {
        double t = 0.0;
        for (int k = 0; k < CL; ++k) t += lds[k * OPW + oi];
        out[o] = t;
        if (h != nullptr && o < hL) {
            const int64_t k = o / B, b = o % B;
            h[(b * nu + k) * (int64_t)nu + n] = t;
        }
    }
}

LaunchInfo launch_reduce(const double* part, int64_t nchunks, int64_t L, double* out, double* h, int B, int nu,
                         int n, hipStream_t s) {
    const int64_t hL = h ? (int64_t)(n + 1) * B : 0;
    LaunchInfo li;
    if (L <= 2048) {
        const int64_t wgs = (L + 3) / 4;
        hipLaunchKernelGGL((k_reduce<4>), dim3(wgs), dim3(WG), 0, s, part, nchunks, L, out, h, B, nu, n, hL);
        li.wgs = wgs;
    } else {
        const int64_t wgs = (L + 15) / 16;
        hipLaunchKernelGGL((k_reduce<16>), dim3(wgs), dim3(WG), 0, s, part, nchunks, L, out, h, B, nu, n, hL);
        li.wgs = wgs;
    }
    li.bytes = (double)(nchunks + 1) * L * 8.0;
    li.flops = (double)nchunks * L;
    return li;
}

// Norm and breakdown of the new residual of each seed (all in FP64):
//   beta = sqrt(w^T S w), eta^2 = |c1|^2 + |c2|^2 + beta^2,
//   breakdown if beta <= tau * eta -> nu_eff = n + 1 and the seed stops;
//   w^T S w < 0 (or not finite) -> nu_eff = -1 (S not positive definite).
__global__ __launch_bounds__(WG) void k_norm(int B, int nk, const double* __restrict__ beta2,
                                             const double* __restrict__ c1, const double* __restrict__ c2,
                                             double tau, int32_t* __restrict__ active, int32_t* __restrict__ nu_eff,
                                             double* __restrict__ beta, int n) {
    // thread (part, b): partial sums of |c1|^2 + |c2|^2 over k = part, part + np, ...
    __shared__ double lds[WG];
    const int np = WG / B;
    const int b = threadIdx.x % B, part = threadIdx.x / B;
    double s = 0.0;
    if (part < np)
        for (int k = part; k < nk; k += np) {
            const double a1 = c1[(int64_t)k * B + b], a2 = c2[(int64_t)k * B + b];
            s += a1 * a1 + a2 * a2;
        }
    lds[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x >= B) return;
    double cc = 0.0;
    for (int q = 0; q < np; ++q) cc += lds[q * B + b];
    if (!active[b]) {
        beta[b] = 0.0;
        return;
    }
    const double bb = beta2[b];
    if (!(bb >= 0.0) || !(bb < INFINITY)) {
        nu_eff[b] = -1;
        active[b] = 0;
        beta[b] = 0.0;
        return;
    }
    const double bt = sqrt(bb);
    const double eta = sqrt(cc + bb);
    if (bt <= tau * eta) {
        nu_eff[b] = n + 1;
        active[b] = 0;
        beta[b] = 0.0;
    } else {
        beta[b] = bt;
    }
}

LaunchInfo launch_norm(int B, int nk, const double* beta2, const double* c1, const double* c2, double tau,
                       int32_t* active, int32_t* nu_eff, double* beta, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_norm, dim3(1), dim3(WG), 0, s, B, nk, beta2, c1, c2, tau, active, nu_eff, beta, n);
    LaunchInfo li;
    li.wgs = 1;
    li.bytes = (2.0 * nk + 3.0) * B * 8.0;
    return li;
}

// out = sum of x[0..n) in a fixed order (strided lane sums, then a tree).
__global__ __launch_bounds__(WG) void k_sum(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
    __shared__ double lds[WG];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += WG) s += x[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int w = WG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = lds[0];
}

LaunchInfo launch_sum(const double* x, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(WG), 0, s, x, n, out);
    LaunchInfo li;
    li.wgs = 1;
    li.bytes = (double)(n + 1) * 8.0;
    return li;
}

// Zero n16 16-byte words (used for the padded rows of the work vectors; a
// kernel rather than a memset so the sequence stays capturable).
__global__ __launch_bounds__(WG) void k_zero(double2* __restrict__ p, int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n16) p[i] = make_double2(0.0, 0.0);
}

LaunchInfo launch_zero(void* p, int64_t bytes, hipStream_t s) {
    const int64_t n16 = bytes / 16;
    const int64_t wgs = (n16 + WG - 1) / WG;
    LaunchInfo li;
    if (wgs > 0) hipLaunchKernelGGL(k_zero, dim3(wgs), dim3(WG), 0, s, (double2*)p, n16);
    li.wgs = wgs;
    li.bytes = (double)bytes;
    return li;
}

}  // namespace mar
