// Subspace eigensolve and Fermi-weighted assembly, one workgroup per seed.
//
// For seed j with m = nu_eff vectors, A = K^T H K (m x m, FP64) is
// diagonalized by the parallel cyclic Jacobi method: each step rotates m / 2
// disjoint index pairs at once (a round-robin tournament, so that every pair
// meets once per sweep of m - 1 steps or m steps for odd m), A <- J^T A J,
// and the same rotations are applied to the rows of the m x (1 + |P(j)|)
// matrix R = [e_1 | K[P(j), :]^T]; sweeps repeat until one rotates nothing.
// No m x m eigenvector matrix is formed. At the end A's diagonal holds the
// levels eps_alpha and row alpha of R holds
//     R[alpha][0]     = y_1alpha            (first component of y_alpha)
//     R[alpha][1 + t] = e_i . v_alpha,  i = P(j)[t],  v_alpha = K y_alpha
// which is all the Green's-function assembly needs (Sec. 2):
//     rho_ij = 2 sum_alpha f_alpha (e_i.v_alpha)(e_j.v_alpha),
//     w_alpha = (e_j^T S v_alpha)(v_alpha^T e_j) = sqrt(S_jj) y_1alpha (e_j.v_alpha)
// (K^T S e_j = sqrt(S_jj) e_1 because u_1 = e_j / sqrt(S_jj) and K^T S K = I),
//     E_j = sum_{i in P(j)} rho_ij H_ij,   N_j = sum_{i in P(j)} rho_ij S_ij.
#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cstdint>

#include "mar_device.h"
#include "mar_internal.h"

namespace mar {

__device__ __forceinline__ double fermi_occ(double eps, double mu, double kT) {
    if (kT == 0.0) return eps < mu ? 1.0 : (eps > mu ? 0.0 : 0.5);
    const double x = (eps - mu) / kT;
    const double t = exp(-fabs(x));
    return x >= 0.0 ? t / (1.0 + t) : 1.0 / (1.0 + t);
}

// Logistic step F(x) = 1/(1+e^-x), and the window of a smoothed delta of width
// sigma over [a, b] (sigma = 0: sharp, 1/2 at an endpoint) for Eq. 3.
__device__ __forceinline__ double logistic_step(double x) {
    const double t = exp(-fabs(x));
    return x >= 0.0 ? 1.0 / (1.0 + t) : t / (1.0 + t);
}
__device__ __forceinline__ double smooth_step(double x, double sigma) {
    if (sigma == 0.0) return x > 0.0 ? 1.0 : (x < 0.0 ? 0.0 : 0.5);
    return logistic_step(x / sigma);
}
__device__ __forceinline__ double level_window(double eps, double a, double b, double sigma) {
    return smooth_step(b - eps, sigma) - smooth_step(a - eps, sigma);
}

// Sum over the 256 threads; every thread gets the same value (butterfly
// pairs add the same two operands, so all lanes agree bit for bit).
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Threads of the eigensolver's workgroup: four waves per SIMD, so that the
// LDS latencies of the Jacobi steps of one seed hide behind each other.
constexpr int EIG_WG = 1024;
constexpr int EIG_WAVES = EIG_WG / 64;
// Per-thread work lists of a Jacobi step when they are short (at most JB blocks
// and JR entries of R per thread, fixed for the whole iteration).
constexpr int JB = 3, JR = 4;

// 1/x and 1/sqrt(x) (x > 0, normal) from the hardware estimates and two Newton steps each (full FP64
// precision: the estimates carry about 23 bits and each step doubles them).
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ double rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// Parallel cyclic Jacobi on the symmetric m x m matrix A (in LDS or global
// memory, upper triangle only: a_ij, i <= j, at A[i * ld + j]; an odd ld spreads
// the column accesses over the LDS banks), each rotation also applied to the
// rows of the m x nr matrix R (R <- J^T R). Run by the whole workgroup.
// Step s of a sweep pairs the indices of a round-robin tournament of n = m
// rounded up to even players (player n - 1 = m is a bye for odd m): position k
// holds players idx(k) and idx(n - 1 - k), idx(0) = 0, idx(i) = 1 + (i - 1 + s)
// mod (n - 1). A pair (p, q) rotates when |a_pq| > eps sqrt(|a_pp a_qq|), with
// the symmetric Schur rotation that zeroes a_pq (tau = (a_qq - a_pp) / (2 a_pq),
// t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1 / sqrt(1 + t^2), s = t c):
// a_pp -= t a_pq, a_qq += t a_pq, a_pq = 0. Every other element belongs to one
// 2 x 2 block of two pairs, J_1^T B J_2, updated in place by one thread (blocks
// k1 <= k2 of pair positions). When the blocks and R's entries make at most JB
// and JR per thread, each thread keeps its list for the whole iteration and
// issues all loads of a step at once; otherwise wave w takes the block rows
// k1 = w, w + 16, ..., its lanes the block columns. Sweeps repeat until one
// rotates nothing, at most max_sweeps. Scratch: cs, sn, tt (n / 2 doubles
// each), cnt (one int). Returns 0 when converged, 1 otherwise. The levels are
// A's diagonal.
__device__ __forceinline__ int jacobi_eig(double* A, int ld, int m, double* R, int nr, double* cs, double* sn,
                                          double* tt, int* cnt, int max_sweeps) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = m + (m & 1), np = n / 2, n1 = n - 1;
    auto off = [&](int i, int j) { return i <= j ? i * ld + j : j * ld + i; };   // a_ij in the upper triangle
    // the pair at position k of step st, p < q (q == m: the bye)
    auto pair = [&](int k, int st, int& p, int& q) {
        int a = k - 1 + st, bb = n - 2 - k + st;
        a = k == 0 ? 0 : 1 + (a >= n1 ? a - n1 : a);
        bb = 1 + (bb >= n1 ? bb - n1 : bb);
        p = a < bb ? a : bb;
        q = a < bb ? bb : a;
    };
    // J_1^T B J_2 on the block of positions k1 < k2 (pairs (p1, q1), (p2, q2)); a bye's row or column is
    // absent (its loads read a_p1p2 again and are dropped)
    auto block = [&](int p1, int q1, double c1, double s1, int p2, int q2, double c2, double s2) {
        const bool hq1 = q1 < m, hq2 = q2 < m, hw = hq1 && hq2;
        const int ox = off(p1, p2);
        const int oy = hq2 ? off(p1, q2) : ox, oz = hq1 ? off(q1, p2) : ox, ow = hw ? off(q1, q2) : ox;
        const double x = A[ox];
        const double y = hq2 ? A[oy] : 0.0, z = hq1 ? A[oz] : 0.0, w = hw ? A[ow] : 0.0;
        const double xr = c1 * x - s1 * z, yr = c1 * y - s1 * w;   // rows: J_1^T B
        const double zr = s1 * x + c1 * z, wr = s1 * y + c1 * w;
        A[ox] = c2 * xr - s2 * yr;                                  // columns: (J_1^T B) J_2
        if (hq2) A[oy] = s2 * xr + c2 * yr;
        if (hq1) A[oz] = c2 * zr - s2 * wr;
        if (hw) A[ow] = s2 * zr + c2 * wr;
    };
    // fixed per-thread lists when short: blocks (k1, k2), k1 <= k2, numbered row by row, and R entries (k, col)
    const int nblk = np * (np + 1) / 2;
    const bool lists = nblk <= JB * EIG_WG && np * nr <= JR * EIG_WG;
    int bk1[JB], bk2[JB], rk[JR], rc[JR];
#pragma unroll
    for (int i = 0; i < JB; ++i) {
        int lin = tid + i * EIG_WG, k1 = 0;
        bk1[i] = -1;
        bk2[i] = 0;
        if (lists && lin < nblk) {
            while (lin >= np - k1) {
                lin -= np - k1;
                ++k1;
            }
            bk1[i] = k1;
            bk2[i] = k1 + lin;
        }
    }
#pragma unroll
    for (int i = 0; i < JR; ++i) {
        const int lin = tid + i * EIG_WG;
        rk[i] = lists && lin < np * nr ? lin / nr : -1;
        rc[i] = lists && lin < np * nr ? lin - (lin / nr) * nr : 0;
    }
    if (tid == 0) *cnt = 0;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        for (int st = 0; st < n1; ++st) {
            // the rotations of this step, one pair per thread
            for (int k = tid; k < np; k += EIG_WG) {
                int p, q;
                pair(k, st, p, q);
                double c = 1.0, sv = 0.0, t = 0.0;
                if (q < m) {
                    const double apq = A[p * ld + q], app = A[p * ld + p], aqq = A[q * ld + q];   // p < q
                    if (apq != 0.0 && apq * apq > (DBL_EPSILON * DBL_EPSILON) * fabs(app * aqq)) {
                        const double tau = (aqq - app) * recip(2.0 * apq);
                        if (fabs(tau) > 1e150) {
                            t = 0.5 * recip(tau);
                        } else {
                            const double r = 1.0 + tau * tau;
                            t = copysign(recip(fabs(tau) + r * rsqrt(r)), tau);
                        }
                        c = rsqrt(1.0 + t * t);
                        sv = t * c;
                        atomicAdd(cnt, 1);
                    }
                }
                cs[k] = c;
                sn[k] = sv;
                tt[k] = t;
            }
            __syncthreads();
            if (lists) {
#pragma unroll
                for (int i = 0; i < JB; ++i) {
                    const int k1 = bk1[i], k2 = bk2[i];
                    if (k1 < 0) continue;
                    int p1, q1;
                    pair(k1, st, p1, q1);
                    const double c1 = cs[k1], s1 = sn[k1];
                    if (k1 == k2) {
                        if (s1 != 0.0) {
                            const double apq = A[p1 * ld + q1], t = tt[k1];
                            A[p1 * ld + p1] -= t * apq;
                            A[q1 * ld + q1] += t * apq;
                            A[p1 * ld + q1] = 0.0;
                        }
                        continue;
                    }
                    const double c2 = cs[k2], s2 = sn[k2];
                    if (s1 == 0.0 && s2 == 0.0) continue;
                    int p2, q2;
                    pair(k2, st, p2, q2);
                    block(p1, q1, c1, s1, p2, q2, c2, s2);
                }
#pragma unroll
                for (int i = 0; i < JR; ++i) {
                    const int k = rk[i], col = rc[i];
                    if (k < 0) continue;
                    const double sv = sn[k];
                    if (sv == 0.0) continue;
                    int p, q;
                    pair(k, st, p, q);
                    const double c = cs[k], rp = R[p * nr + col], rq = R[q * nr + col];
                    R[p * nr + col] = c * rp - sv * rq;
                    R[q * nr + col] = sv * rp + c * rq;
                }
            } else {
                for (int k1 = wave; k1 < np; k1 += EIG_WAVES) {
                    int p1, q1;
                    pair(k1, st, p1, q1);
                    const double c1 = cs[k1], s1 = sn[k1];
                    for (int k2 = k1 + lane; k2 < np; k2 += 64) {
                        if (k2 == k1) {
                            if (s1 != 0.0) {
                                const double apq = A[p1 * ld + q1], t = tt[k1];
                                A[p1 * ld + p1] -= t * apq;
                                A[q1 * ld + q1] += t * apq;
                                A[p1 * ld + q1] = 0.0;
                            }
                            continue;
                        }
                        const double c2 = cs[k2], s2 = sn[k2];
                        if (s1 == 0.0 && s2 == 0.0) continue;
                        int p2, q2;
                        pair(k2, st, p2, q2);
                        block(p1, q1, c1, s1, p2, q2, c2, s2);
                    }
                }
                for (int k = wave; k < np; k += EIG_WAVES) {
                    const double sv = sn[k];
                    if (sv == 0.0) continue;
                    int p, q;
                    pair(k, st, p, q);
                    const double c = cs[k];
                    for (int col = lane; col < nr; col += 64) {
                        const double rp = R[p * nr + col], rq = R[q * nr + col];
                        R[p * nr + col] = c * rp - sv * rq;
                        R[q * nr + col] = sv * rp + c * rq;
                    }
                }
            }
            __syncthreads();
        }
        const int rotated = *cnt;
        __syncthreads();
        if (tid == 0) *cnt = 0;
        __syncthreads();
        if (rotated == 0) return 0;
    }
    return 1;
}

size_t eig_lds_bytes(int nu, int max_row, bool a_in_lds) {
    size_t n = (a_in_lds ? (size_t)nu * (nu + 1) : 0) + (size_t)nu * (max_row + 1) + 4 * (size_t)nu + 8 + 72 + 64 + 2;
    return n * sizeof(double);
}

bool eig_a_fits_lds(int nu, int max_row) { return eig_lds_bytes(nu, max_row, true) <= 160 * 1024; }

// Rows K[P(j), :] of each seed, gathered from the seed-interleaved basis into
// Kp[(b * nu + k) * max_row + t] (FP64), with the seed's nu_eff copied beside
// them, so that the eigensolve can run while the basis is reused.
template <typename T>
__global__ __launch_bounds__(WG) void k_gather_rows(int nseeds, const int32_t* __restrict__ seeds, int B, int nu,
                                                    const int32_t* __restrict__ nu_eff_blk, const T* __restrict__ K,
                                                    int64_t stride, const int32_t* __restrict__ Hrp,
                                                    const int32_t* __restrict__ Hcol, int max_row,
                                                    double* __restrict__ Kp, int32_t* __restrict__ nu_copy) {
    const int b = blockIdx.x;
    if (b >= nseeds) return;
    const int m = nu_eff_blk[b];
    if (threadIdx.x == 0) nu_copy[b] = m;
    if (m <= 0) return;
    const int j = seeds[b];
    const int rlo = Hrp[j], nP = Hrp[j + 1] - rlo;
    for (int idx = threadIdx.x; idx < m * nP; idx += WG) {
        const int k = idx / nP, t = idx - k * nP;
        Kp[((int64_t)b * nu + k) * max_row + t] = (double)K[(int64_t)k * stride + (int64_t)Hcol[rlo + t] * B + b];
    }
}

template <bool LDS_A>
__global__ __launch_bounds__(EIG_WG) void k_eig(EigExtra ex, int nseeds, const int32_t* __restrict__ seeds, int nu,
                                            double* __restrict__ h, const int32_t* __restrict__ nu_eff_blk,
                                            const double* __restrict__ Kp, const int32_t* __restrict__ Hrp,
                                            const int32_t* __restrict__ Hcol, const double* __restrict__ Hval,
                                            const double* __restrict__ SvalH, const double* __restrict__ diagS,
                                            int max_row, double mu, double kT, double* __restrict__ rho,
                                            double* __restrict__ e_seed, double* __restrict__ n_seed,
                                            int32_t* __restrict__ nu_eff_out, double* __restrict__ eps_out,
                                            double* __restrict__ w_out, double* __restrict__ zc) {
    extern __shared__ double smem[];
    const int b = blockIdx.x;
    if (b >= nseeds) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = nu_eff_blk[b];
    double* eps_b = eps_out ? eps_out + (int64_t)b * nu : nullptr;
    double* w_b = w_out ? w_out + (int64_t)b * nu : nullptr;
    if (m <= 0) {
        if (tid == 0) {
            nu_eff_out[b] = m;
            e_seed[b] = 0.0;
            n_seed[b] = 0.0;
        }
        for (int a = tid; a < nu; a += EIG_WG) {
            if (eps_b) eps_b[a] = 0.0;
            if (w_b) w_b[a] = 0.0;
        }
        return;
    }
    const int j = seeds[b];
    const int rlo = Hrp[j];
    const int nP = Hrp[j + 1] - rlo;
    // columns of R: [e_1 | K[P(j),:]^T] (+ [K^T v_ref] in mode 2), or [e_1 | I_m] in mode 1
    const int NR = ex.mode == 1 ? m + 1 : (ex.mode == 2 ? nP + 2 : nP + 1);

    double* A;
    int ld;
    double* p = smem;
    if constexpr (LDS_A) {
        A = p;
        ld = m | 1;   // odd: the Jacobi steps' column accesses spread over the banks
        p += (size_t)nu * (nu + 1);
    } else {
        A = h + (int64_t)b * nu * nu;
        ld = nu;
    }
    double* Rl = p;
    double* R = ex.mode == 1 ? ex.Rg + (int64_t)b * nu * (nu + 1) : Rl;
    p += (size_t)nu * (max_row + (ex.mode == 2 ? 2 : 1));
    double* d = p;
    p += nu;
    double* e = p;
    p += nu;
    double* v = p;
    p += nu;
    double* q = p;
    p += nu;
    double* red = p;
    p += 8;
    p += 72;
    double* rhoL = p;
    p += 64;
    int* tjp = reinterpret_cast<int*>(p);

    // A = K^T H K from its computed upper triangle (h[b][k][n], k <= n), which is all the Jacobi
    // iteration keeps (in place in h when A does not fit in LDS).
    const double* hb = h + (int64_t)b * nu * nu;
    if constexpr (LDS_A) {
        for (int r = wave; r < m; r += EIG_WAVES)
            for (int c = r + lane; c < m; c += 64) A[r * ld + c] = hb[(int64_t)r * nu + c];
    }
    for (int idx = tid; idx < m * NR; idx += EIG_WG) {
        const int k = idx / NR, c = idx - k * NR;
        double r0;
        if (c == 0) r0 = k == 0 ? 1.0 : 0.0;
        else if (ex.mode == 1) r0 = k == c - 1 ? 1.0 : 0.0;
        else if (c <= nP) r0 = Kp[((int64_t)b * nu + k) * max_row + (c - 1)];
        else r0 = ex.pref[(int64_t)k * ex.pB + b];
        R[idx] = r0;
    }
    if (tid < nP && Hcol[rlo + tid] == j) *tjp = tid;
    __syncthreads();

    // Jacobi: A's diagonal becomes the levels, R's rows the vectors' components (cs, sn, tt in v, q, e)
    int* failp = tjp + 1;
    {
        // a separate call for R in global memory (mode 1), so that the LDS case compiles to LDS instructions
        const int f = ex.mode == 1 ? jacobi_eig(A, ld, m, R, NR, v, q, e, tjp + 2, ex.eig_max_sweeps)
                                   : jacobi_eig(A, ld, m, Rl, NR, v, q, e, tjp + 2, ex.eig_max_sweeps);
        __syncthreads();
        for (int a = tid; a < m; a += EIG_WG) d[a] = A[a * ld + a];
        if (tid == 0) *failp = f;
    }
    __syncthreads();
    if (*failp != 0) {
        // an eigenvalue is still unconverged: the seed reports NU_NOCONV and NaN in every output
        const double nan = __builtin_nan("");
        if (ex.mode == 1) {
            for (int idx = tid; idx < m * m; idx += EIG_WG) {
                const int a = idx / m, c = idx - a * m;
                ex.Y[((int64_t)b * nu + a) * nu + c] = nan;
            }
        } else if (ex.mode == 2) {
            if (tid == 0) ex.phi[b] = nan;
        } else if (zc == nullptr) {
            for (int t = tid; t < nP; t += EIG_WG) rho[rlo + t] = nan;
            if (tid == 0) {
                e_seed[b] = nan;
                n_seed[b] = nan;
            }
        }
        for (int a = tid; a < nu; a += EIG_WG) {
            if (eps_b) eps_b[a] = nan;
            if (w_b) w_b[a] = nan;
        }
        if (tid == 0) nu_eff_out[b] = NU_NOCONV;
        return;
    }

    // Fermi-weighted assembly, or (zc != nullptr) keep the rows e_i.v_alpha,
    // i in P(j), for an assembly at a Fermi level found later (k_assemble).
    const int tj = *tjp;
    const double sq = sqrt(diagS[j]);
    if (ex.mode == 1) {   // the full subspace eigenvectors y_alpha and levels
        for (int idx = tid; idx < m * m; idx += EIG_WG) {
            const int a = idx / m, c = idx - a * m;
            ex.Y[((int64_t)b * nu + a) * nu + c] = R[a * NR + 1 + c];
        }
        for (int a = tid; a < nu; a += EIG_WG) eps_b[a] = a < m ? d[a] : 0.0;
        if (tid == 0) nu_eff_out[b] = m;
        return;
    }
    if (ex.mode == 2) {   // Eq. 3 with the inner-product signs: sum_alpha s_alpha (e_j.v_alpha) window_alpha
        if (tid == 0) {
            const double lo = ex.win[1], hi = ex.win[2];
            double phi = 0.0;
            for (int a = 0; a < m; ++a) {
                const double c = R[a * NR + 1 + tj] * level_window(d[a], lo, hi, ex.sigma);
                phi += R[a * NR + NR - 1] >= 0.0 ? c : -c;
            }
            ex.phi[b] = phi;
            nu_eff_out[b] = m;
        }
        return;
    }
    if (zc != nullptr) {
        double* zb = zc + (int64_t)b * nu * max_row;
        for (int idx = tid; idx < m * nP; idx += EIG_WG) {
            const int a = idx / nP, t = idx - a * nP;
            zb[a * max_row + t] = R[a * NR + 1 + t];
        }
        for (int a = tid; a < m; a += EIG_WG) {
            eps_b[a] = d[a];
            w_b[a] = sq * R[a * NR] * R[a * NR + 1 + tj];
        }
        for (int a = m + tid; a < nu; a += EIG_WG) {
            eps_b[a] = 0.0;
            w_b[a] = 0.0;
        }
        if (tid == 0) nu_eff_out[b] = m;
        return;
    }
    double* fz = q;
    for (int a = tid; a < m; a += EIG_WG) {
        const double ea = d[a];
        const double zj = R[a * NR + 1 + tj];
        fz[a] = fermi_occ(ea, mu, kT) * zj;
        if (eps_b) eps_b[a] = ea;
        if (w_b) w_b[a] = sq * R[a * NR] * zj;
    }
    for (int a = m + tid; a < nu; a += EIG_WG) {
        if (eps_b) eps_b[a] = 0.0;
        if (w_b) w_b[a] = 0.0;
    }
    __syncthreads();
    for (int cb = 0; cb < nP; cb += EIG_WG / 8) {
        const int t = cb + (tid >> 3), pi = tid & 7;
        double s = 0.0;
        if (t < nP)
            for (int a = pi; a < m; a += 8) s += fz[a] * R[a * NR + 1 + t];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        if (t < nP && pi == 0) {
            const double r = 2.0 * s;
            rho[rlo + t] = r;
            rhoL[t] = r;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double E = 0.0, N = 0.0;
        for (int t = 0; t < nP; ++t) {
            E += rhoL[t] * Hval[rlo + t];
            N += rhoL[t] * SvalH[rlo + t];
        }
        e_seed[b] = E;
        n_seed[b] = N;
        nu_eff_out[b] = m;
    }
}

// Lets kernel f use up to 160 KB of dynamic LDS. The attribute belongs to the current device, so it is
// set once per device (bit d of done for device d; concurrent first calls both set it, which is harmless).
static void allow_full_lds(const void* f, std::atomic<uint64_t>& done) {
    int dev = 0;
    const bool known = hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64;
    const uint64_t bit = known ? 1ull << dev : 0;
    if (known && (done.load(std::memory_order_acquire) & bit)) return;
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (known) done.fetch_or(bit, std::memory_order_acq_rel);
}

LaunchInfo launch_eig(int nseeds, const int32_t* seeds, int nu, double* h, const int32_t* nu_eff_blk,
                      const double* Kp, const int32_t* Hrp, const int32_t* Hcol, const double* Hval,
                      const double* SvalH, const double* diagS, int max_row, double mu, double kT, double* rho,
                      double* e_seed, double* n_seed, int32_t* nu_eff_out, double* eps_out, double* w_out,
                      double* zc, const EigExtra& ex, hipStream_t s) {
    const int rcols = max_row + (ex.mode == 2 ? 1 : 0);   // R's LDS share (mode 1 keeps R in global memory)
    const bool lds_a = eig_a_fits_lds(nu, rcols);
    const size_t lds = eig_lds_bytes(nu, rcols, lds_a);
    if (lds_a) {
        static std::atomic<uint64_t> done{0};
        allow_full_lds((const void*)k_eig<true>, done);
        hipLaunchKernelGGL((k_eig<true>), dim3(nseeds), dim3(EIG_WG), lds, s, ex, nseeds, seeds, nu, h, nu_eff_blk, Kp, Hrp,
                           Hcol, Hval, SvalH, diagS, max_row, mu, kT, rho, e_seed, n_seed, nu_eff_out, eps_out, w_out,
                           zc);
    } else {
        static std::atomic<uint64_t> done{0};
        allow_full_lds((const void*)k_eig<false>, done);
        hipLaunchKernelGGL((k_eig<false>), dim3(nseeds), dim3(EIG_WG), lds, s, ex, nseeds, seeds, nu, h, nu_eff_blk, Kp,
                           Hrp, Hcol, Hval, SvalH, diagS, max_row, mu, kT, rho, e_seed, n_seed, nu_eff_out, eps_out,
                           w_out, zc);
    }
    LaunchInfo li;
    li.wgs = nseeds;
    const double nv = (double)nu;
    li.bytes = (double)nseeds * (nv * nv * 8.0 + nv * max_row * 8.0 + (max_row + 3) * 8.0 * 3);
    li.flops = (double)nseeds * ((4.0 / 3.0) * nv * nv * nv + 4.0 * nv * nv * (max_row + 1));
    return li;
}

// ---------------------------------------------------------------------------
// Assembly at a Fermi level held on the device (after k_eig with zc != nullptr):
// the same sums, in the same order, as the fused epilogue of k_eig.
__global__ __launch_bounds__(WG) void k_assemble(int nseeds, const int32_t* __restrict__ seeds, int nu,
                                                 const int32_t* __restrict__ nu_eff, const double* __restrict__ eps,
                                                 const double* __restrict__ zc, int max_row,
                                                 const int32_t* __restrict__ Hrp, const int32_t* __restrict__ Hcol,
                                                 const double* __restrict__ Hval, const double* __restrict__ SvalH,
                                                 const double* __restrict__ mu_p, double kT, double* __restrict__ rho,
                                                 double* __restrict__ e_seed, double* __restrict__ n_seed) {
    __shared__ double fz[MAX_NU_ASSEMBLE];
    __shared__ double rhoL[64];
    __shared__ int tjs;
    const int b = blockIdx.x, tid = threadIdx.x;
    if (b >= nseeds) return;
    const int m = nu_eff[b];
    if (m <= 0) {
        // a seed whose subspace eigensolve did not converge gets NaN outputs, as in k_eig
        const double fill = m == NU_NOCONV ? __builtin_nan("") : 0.0;
        if (m == NU_NOCONV)
            for (int t = Hrp[seeds[b]] + tid; t < Hrp[seeds[b] + 1]; t += WG) rho[t] = fill;
        if (tid == 0) {
            e_seed[b] = fill;
            n_seed[b] = fill;
        }
        return;
    }
    const int j = seeds[b];
    const int rlo = Hrp[j], nP = Hrp[j + 1] - rlo;
    if (tid < nP && Hcol[rlo + tid] == j) tjs = tid;
    __syncthreads();
    const int tj = tjs;
    const double mu = *mu_p;
    const double* zb = zc + (int64_t)b * nu * max_row;
    for (int a = tid; a < m; a += WG) fz[a] = fermi_occ(eps[(int64_t)b * nu + a], mu, kT) * zb[a * max_row + tj];
    __syncthreads();
    for (int cb = 0; cb < nP; cb += WG / 8) {
        const int t = cb + (tid >> 3), pi = tid & 7;
        double s = 0.0;
        if (t < nP)
            for (int a = pi; a < m; a += 8) s += fz[a] * zb[a * max_row + t];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        if (t < nP && pi == 0) {
            const double r = 2.0 * s;
            rho[rlo + t] = r;
            rhoL[t] = r;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double E = 0.0, N = 0.0;
        for (int t = 0; t < nP; ++t) {
            E += rhoL[t] * Hval[rlo + t];
            N += rhoL[t] * SvalH[rlo + t];
        }
        e_seed[b] = E;
        n_seed[b] = N;
    }
}

LaunchInfo launch_assemble(int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff, const double* eps,
                           const double* zc, int max_row, const int32_t* Hrp, const int32_t* Hcol,
                           const double* Hval, const double* SvalH, const double* mu, double kT, double* rho,
                           double* e_seed, double* n_seed, hipStream_t s) {
    LaunchInfo li;
    if (nu > MAX_NU_ASSEMBLE || max_row > 64) {
        li.wgs = -1;
        return li;
    }
    if (nseeds > 0)
        hipLaunchKernelGGL(k_assemble, dim3(nseeds), dim3(WG), 0, s, nseeds, seeds, nu, nu_eff, eps, zc, max_row, Hrp,
                           Hcol, Hval, SvalH, mu, kT, rho, e_seed, n_seed);
    li.wgs = nseeds;
    li.bytes = (double)nseeds * ((double)nu * (max_row + 1) * 8.0 + 3.0 * max_row * 8.0);
    li.flops = (double)nseeds * 2.0 * nu * (max_row + 1);
    return li;
}

// ---------------------------------------------------------------------------
// Fermi level on the device: mu with N(mu) = sum_j 2 sum_alpha f((eps_alpha^(j)
// - mu)/kT) w_alpha^(j) equal to n_target, by bisection on [min eps - 40 kT,
// max eps + 40 kT] over the listed seeds' subspace levels (alpha < nu_eff).
// st = {lo, hi, mu}. Every sum runs in a fixed order.
constexpr int MU_WGS = 512;   // workgroups of the counting kernel

__device__ __forceinline__ void wg_minmax(double& lo, double& hi, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off));
        hi = fmax(hi, __shfl_xor(hi, off));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[wave] = lo;
        red[4 + wave] = hi;
    }
    __syncthreads();
    lo = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
    hi = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
}

__global__ __launch_bounds__(WG) void k_mu_bounds(int64_t nseeds, int nu, const int32_t* __restrict__ nu_eff,
                                                  const double* __restrict__ eps, double* __restrict__ part) {
    __shared__ double red[8];
    double lo = INFINITY, hi = -INFINITY;
    const int64_t npair = nseeds * nu;
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < npair; p += (int64_t)gridDim.x * WG) {
        const int64_t b = p / nu;
        const int a = (int)(p - b * nu);
        if (a < nu_eff[b]) {
            lo = fmin(lo, eps[p]);
            hi = fmax(hi, eps[p]);
        }
    }
    wg_minmax(lo, hi, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = lo;
        part[2 * blockIdx.x + 1] = hi;
    }
}

__global__ __launch_bounds__(64) void k_mu_init(int nwg, const double* __restrict__ part, double kT,
                                                double* __restrict__ st) {
    if (threadIdx.x != 0) return;
    double lo = INFINITY, hi = -INFINITY;
    for (int g = 0; g < nwg; ++g) {
        lo = fmin(lo, part[2 * g]);
        hi = fmax(hi, part[2 * g + 1]);
    }
    if (!(lo <= hi)) lo = hi = 0.0;   // no levels at all
    st[0] = lo - 40.0 * kT;
    st[1] = hi + 40.0 * kT;
    st[2] = 0.5 * (st[0] + st[1]);
}

__global__ __launch_bounds__(WG) void k_mu_count(int64_t nseeds, int nu, const int32_t* __restrict__ nu_eff,
                                                 const double* __restrict__ eps, const double* __restrict__ w,
                                                 double kT, const double* __restrict__ st, double* __restrict__ part) {
    __shared__ double red[8];
    const double mid = 0.5 * (st[0] + st[1]);
    double s = 0.0;
    const int64_t npair = nseeds * nu;
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < npair; p += (int64_t)gridDim.x * WG) {
        const int64_t b = p / nu;
        const int a = (int)(p - b * nu);
        if (a < nu_eff[b]) s += 2.0 * fermi_occ(eps[p], mid, kT) * w[p];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(64) void k_mu_step(int nwg, const double* __restrict__ part, double n_target,
                                                double* __restrict__ st, int last, double* __restrict__ mu_out) {
    if (threadIdx.x != 0) return;
    double n = 0.0;
    for (int g = 0; g < nwg; ++g) n += part[g];
    const double mid = 0.5 * (st[0] + st[1]);
    if (n < n_target) st[0] = mid;
    else st[1] = mid;
    if (last) {
        st[2] = 0.5 * (st[0] + st[1]);
        if (mu_out) *mu_out = st[2];
    }
}

LaunchInfo launch_fermi_search(int64_t nseeds, int nu, const int32_t* nu_eff, const double* eps, const double* w,
                               double n_target, double kT, int iters, double* part, double* st, double* mu_out,
                               hipStream_t s) {
    const int64_t npair = nseeds * nu;
    int nwg = (int)std::min<int64_t>(MU_WGS, std::max<int64_t>(1, (npair + WG - 1) / WG));
    hipLaunchKernelGGL(k_mu_bounds, dim3(nwg), dim3(WG), 0, s, nseeds, nu, nu_eff, eps, part);
    hipLaunchKernelGGL(k_mu_init, dim3(1), dim3(64), 0, s, nwg, part, kT, st);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_mu_count, dim3(nwg), dim3(WG), 0, s, nseeds, nu, nu_eff, eps, w, kT, st, part);
        hipLaunchKernelGGL(k_mu_step, dim3(1), dim3(64), 0, s, nwg, part, n_target, st, it + 1 == iters ? 1 : 0,
                           mu_out);
    }
    LaunchInfo li;
    li.wgs = nwg;
    li.bytes = (double)(iters + 1) * npair * 20.0;
    li.flops = (double)iters * npair * 30.0;
    return li;
}

// ---------------------------------------------------------------------------
// Eigen states (Sec. 3, Eq. 3; Appendix): integrated density of states
//   n(eta) = sum_j sum_alpha w_alpha^(j) F((eta - eps_alpha^(j)) / sigma)
// (F the logistic step; sigma = 0: the unit step, 1/2 at 0), bisected for the
// three counts k - 1, k - 1/2 and k at once on [min eps - 1, max eps + 1].
// st = {lo, hi} x 3; lv = {eta(k - 1/2), eta(k - 1), eta(k)}.
__global__ __launch_bounds__(64) void k_dos_init(int nwg, const double* __restrict__ part, double* __restrict__ st) {
    if (threadIdx.x != 0) return;
    double lo = INFINITY, hi = -INFINITY;
    for (int g = 0; g < nwg; ++g) {
        lo = fmin(lo, part[2 * g]);
        hi = fmax(hi, part[2 * g + 1]);
    }
    if (!(lo <= hi)) lo = hi = 0.0;
    for (int t = 0; t < 3; ++t) {
        st[2 * t] = lo - 1.0;
        st[2 * t + 1] = hi + 1.0;
    }
}

__global__ __launch_bounds__(WG) void k_dos_count(int64_t nseeds, int nu, const int32_t* __restrict__ nu_eff,
                                                  const double* __restrict__ eps, const double* __restrict__ w,
                                                  double sigma, const double* __restrict__ st,
                                                  double* __restrict__ part) {
    __shared__ double red[8];
    double mid[3], c[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 3; ++t) mid[t] = 0.5 * (st[2 * t] + st[2 * t + 1]);
    const int64_t npair = nseeds * nu;
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < npair; p += (int64_t)gridDim.x * WG) {
        const int64_t b = p / nu;
        const int a = (int)(p - b * nu);
        if (a < nu_eff[b]) {
#pragma unroll
            for (int t = 0; t < 3; ++t) c[t] += w[p] * smooth_step(mid[t] - eps[p], sigma);
        }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const double v = block_sum(c[t], red);
        if (threadIdx.x == 0) part[3 * blockIdx.x + t] = v;
    }
}

__global__ __launch_bounds__(64) void k_dos_step(int nwg, const double* __restrict__ part, int k,
                                                 double* __restrict__ st, int last, double* __restrict__ lv) {
    if (threadIdx.x != 0) return;
    const double target[3] = {k - 1.0, k - 0.5, (double)k};
    for (int t = 0; t < 3; ++t) {
        double n = 0.0;
        for (int g = 0; g < nwg; ++g) n += part[3 * g + t];
        const double mid = 0.5 * (st[2 * t] + st[2 * t + 1]);
        if (n < target[t]) st[2 * t] = mid;
        else st[2 * t + 1] = mid;
    }
    if (last) {
        lv[0] = 0.5 * (st[2] + st[3]);   // eps_k = eta(k - 1/2)
        lv[1] = 0.5 * (st[0] + st[1]);   // eta(k - 1)
        lv[2] = 0.5 * (st[4] + st[5]);   // eta(k)
    }
}

LaunchInfo launch_dos_search(int64_t nseeds, int nu, const int32_t* nu_eff, const double* eps, const double* w,
                             double sigma, int k, int iters, double* part, double* st, double* lv, hipStream_t s) {
    const int64_t npair = nseeds * nu;
    const int nwg = (int)std::min<int64_t>(MU_WGS, std::max<int64_t>(1, (npair + WG - 1) / WG));
    hipLaunchKernelGGL(k_mu_bounds, dim3(nwg), dim3(WG), 0, s, nseeds, nu, nu_eff, eps, part);
    hipLaunchKernelGGL(k_dos_init, dim3(1), dim3(64), 0, s, nwg, part, st);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_dos_count, dim3(nwg), dim3(WG), 0, s, nseeds, nu, nu_eff, eps, w, sigma, st, part);
        hipLaunchKernelGGL(k_dos_step, dim3(1), dim3(64), 0, s, nwg, part, k, st, it + 1 == iters ? 1 : 0, lv);
    }
    LaunchInfo li;
    li.wgs = nwg;
    li.bytes = (double)(iters + 1) * npair * 20.0;
    li.flops = (double)iters * npair * 90.0;
    return li;
}

// Contributions c_alpha^(j) = (e_j . v_alpha^(j)) window_alpha of every seed
// (kept rows zc, levels eps) and the reference: the largest |c| (first seed,
// then first alpha, on ties). ref = {position b, alpha, seed j}; refseed[0] = j.
__global__ __launch_bounds__(WG) void k_es_contrib(int nseeds, const int32_t* __restrict__ seeds, int nu,
                                                   const int32_t* __restrict__ nu_eff, const double* __restrict__ eps,
                                                   const double* __restrict__ zc, int max_row,
                                                   const int32_t* __restrict__ Hrp, const int32_t* __restrict__ Hcol,
                                                   const double* __restrict__ lv, double sigma,
                                                   double* __restrict__ cmax, int32_t* __restrict__ amax) {
    __shared__ int tjs;
    const int b = blockIdx.x;
    if (b >= nseeds) return;
    const int m = nu_eff[b];
    if (m <= 0) {
        if (threadIdx.x == 0) {
            cmax[b] = -1.0;
            amax[b] = 0;
        }
        return;
    }
    const int j = seeds[b];
    const int rlo = Hrp[j], nP = Hrp[j + 1] - rlo;
    if ((int)threadIdx.x < nP && Hcol[rlo + threadIdx.x] == j) tjs = threadIdx.x;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double* zb = zc + (int64_t)b * nu * max_row;
    double best = -1.0;
    int ba = 0;
    for (int a = 0; a < m; ++a) {
        const double c = fabs(zb[a * max_row + tjs] * level_window(eps[(int64_t)b * nu + a], lv[1], lv[2], sigma));
        if (c > best) {
            best = c;
            ba = a;
        }
    }
    cmax[b] = best;
    amax[b] = ba;
}

__global__ __launch_bounds__(64) void k_es_argmax(int nseeds, const int32_t* __restrict__ seeds,
                                                  const double* __restrict__ cmax, const int32_t* __restrict__ amax,
                                                  int32_t* __restrict__ ref, int32_t* __restrict__ refseed) {
    if (threadIdx.x != 0) return;
    double best = -1.0;
    int bb = 0;
    for (int b = 0; b < nseeds; ++b)
        if (cmax[b] > best) {
            best = cmax[b];
            bb = b;
        }
    ref[0] = bb;
    ref[1] = nseeds > 0 ? amax[bb] : 0;
    ref[2] = nseeds > 0 ? seeds[bb] : 0;
    refseed[0] = ref[2];
}

LaunchInfo launch_es_reference(int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff, const double* eps,
                               const double* zc, int max_row, const int32_t* Hrp, const int32_t* Hcol,
                               const double* lv, double sigma, double* cmax, int32_t* amax, int32_t* ref,
                               int32_t* refseed, hipStream_t s) {
    if (nseeds > 0)
        hipLaunchKernelGGL(k_es_contrib, dim3(nseeds), dim3(WG), 0, s, nseeds, seeds, nu, nu_eff, eps, zc, max_row, Hrp,
                           Hcol, lv, sigma, cmax, amax);
    hipLaunchKernelGGL(k_es_argmax, dim3(1), dim3(64), 0, s, nseeds, seeds, cmax, amax, ref, refseed);
    LaunchInfo li;
    li.wgs = nseeds;
    li.bytes = (double)nseeds * nu * 16.0;
    return li;
}

// Reference seed (solved alone, B = 1): pick among its subspace eigenvectors
// the one with the largest |(e_j . v_alpha) window_alpha| (v_alpha = K y_alpha),
// and form v_ref = K y_ref over all rows.
template <typename T>
__global__ __launch_bounds__(WG) void k_es_pick(const T* __restrict__ K, int64_t stride, const int32_t* __restrict__ seed,
                                                int nu, const int32_t* __restrict__ nu_eff,
                                                const double* __restrict__ Y, const double* __restrict__ eps,
                                                const double* __restrict__ lv, double sigma,
                                                double* __restrict__ yref) {
    __shared__ double cs[WG];
    __shared__ int as[WG];
    const int m = nu_eff[0];
    const int j = seed[0];
    double best = -1.0;
    int ba = 0;
    for (int a = threadIdx.x; a < m; a += WG) {
        double z = 0.0;
        for (int k = 0; k < m; ++k) z += (double)K[(int64_t)k * stride + j] * Y[(int64_t)a * nu + k];
        const double c = fabs(z * level_window(eps[a], lv[1], lv[2], sigma));
        if (c > best) {
            best = c;
            ba = a;
        }
    }
    cs[threadIdx.x] = best;
    as[threadIdx.x] = ba;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int t = 1; t < WG; ++t)
        if (cs[t] > best || (cs[t] == best && as[t] < ba)) {
            best = cs[t];
            ba = as[t];
        }
    for (int k = 0; k < nu; ++k) yref[k] = k < m ? Y[(int64_t)ba * nu + k] : 0.0;
}

template <typename T>
__global__ __launch_bounds__(WG) void k_es_vref(const T* __restrict__ K, int64_t stride, int64_t M, int nu,
                                                const int32_t* __restrict__ nu_eff, const double* __restrict__ yref,
                                                double* __restrict__ vref) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= M) return;
    const int m = nu_eff[0];
    double v = 0.0;
    for (int k = 0; k < m; ++k) v += (double)K[(int64_t)k * stride + i] * yref[k];
    vref[i] = v;
}

template <typename T>
LaunchInfo launch_es_refvec(const T* K, int64_t stride, int64_t M, const int32_t* seed, int nu,
                            const int32_t* nu_eff, const double* Y, const double* eps, const double* lv, double sigma,
                            double* yref, double* vref, hipStream_t s) {
    hipLaunchKernelGGL((k_es_pick<T>), dim3(1), dim3(WG), 0, s, K, stride, seed, nu, nu_eff, Y, eps, lv, sigma, yref);
    const int64_t wgs = (M + WG - 1) / WG;
    hipLaunchKernelGGL((k_es_vref<T>), dim3((unsigned)wgs), dim3(WG), 0, s, K, stride, M, nu, nu_eff, yref, vref);
    LaunchInfo li;
    li.wgs = wgs;
    li.bytes = (double)nu * M * (sizeof(T) + 8.0 / nu);
    return li;
}
template LaunchInfo launch_es_refvec<float>(const float*, int64_t, int64_t, const int32_t*, int, const int32_t*,
                                            const double*, const double*, const double*, double, double*, double*,
                                            hipStream_t);
template LaunchInfo launch_es_refvec<double>(const double*, int64_t, int64_t, const int32_t*, int, const int32_t*,
                                             const double*, const double*, const double*, double, double*, double*,
                                             hipStream_t);

template <typename T>
static LaunchInfo launch_gather_t(int B, int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff_blk,
                                  const T* K, int64_t stride, const int32_t* Hrp, const int32_t* Hcol, int max_row,
                                  double* Kp, int32_t* nu_copy, hipStream_t s) {
    hipLaunchKernelGGL((k_gather_rows<T>), dim3(nseeds), dim3(WG), 0, s, nseeds, seeds, B, nu, nu_eff_blk, K, stride, Hrp,
                       Hcol, max_row, Kp, nu_copy);
    LaunchInfo li;
    li.wgs = nseeds;
    li.bytes = (double)nseeds * nu * max_row * (sizeof(T) + 8.0);
    return li;
}

template <>
LaunchInfo launch_gather<float>(int B, int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff_blk,
                                const float* K, int64_t stride, const int32_t* Hrp, const int32_t* Hcol, int max_row,
                                double* Kp, int32_t* nu_copy, hipStream_t s) {
    return launch_gather_t<float>(B, nseeds, seeds, nu, nu_eff_blk, K, stride, Hrp, Hcol, max_row, Kp, nu_copy, s);
}

template <>
LaunchInfo launch_gather<double>(int B, int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff_blk,
                                 const double* K, int64_t stride, const int32_t* Hrp, const int32_t* Hcol, int max_row,
                                 double* Kp, int32_t* nu_copy, hipStream_t s) {
    return launch_gather_t<double>(B, nseeds, seeds, nu, nu_eff_blk, K, stride, Hrp, Hcol, max_row, Kp, nu_copy, s);
}

}  // namespace mar
