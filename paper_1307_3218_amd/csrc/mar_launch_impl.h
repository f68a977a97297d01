// Streaming kernels of the Krylov/CGS2 phase and their launchers, for one
// element type MAR_T (float or double). Included once per type.
//
// Layout (all per seed block of B seeds): vectors are [M][B] with the seed
// index fastest; the basis K and S*K are [nu][M][B] (slab k = k-th vector of
// every seed). Each kernel streams whole slabs with 16-byte vector accesses.
#include <type_traits>

#include "mar_device.h"
#include "mar_internal.h"

#ifndef MAR_T
#error "define MAR_T before including"
#endif

namespace mar {

// ---------------------------------------------------------------------------
// u_1 = e_j / sqrt(S_jj) for every seed of the block (the first basis vector,
// which puts e_j in L_nu^(j)); flags seeds outside [0, M) as invalid.
template <typename T, int B>
__global__ __launch_bounds__(WG) void k_init(int64_t Mp, int64_t M, const int32_t* __restrict__ seeds, int nseeds,
                                             const double* __restrict__ diagS, int nu, T* __restrict__ K0,
                                             int32_t* __restrict__ active, int32_t* __restrict__ nu_eff,
                                             double* __restrict__ uu) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC;
    using VT = typename Vec16<T>::type;
    const int64_t nvec = Mp * B / VEC;
    const int64_t vi = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (vi < B) {
        const int b = (int)vi;
        const int j = b < nseeds ? seeds[b] : -1;
        const bool ok = j >= 0 && j < M;
        active[b] = ok ? 1 : 0;
        nu_eff[b] = ok ? nu : (b < nseeds ? -2 : 0);
        if (uu) uu[b] = ok ? 1.0 / diagS[j] : 0.0;   // u_1 . u_1
    }
    if (vi >= nvec) return;
    T a[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
        const int64_t e = vi * VEC + i;
        const int64_t row = e / B;
        const int b = (int)(e % B);
        const int j = b < nseeds ? seeds[b] : -1;
        a[i] = (j >= 0 && j < M && row == j) ? (T)(1.0 / sqrt(diagS[j])) : (T)0;
    }
    reinterpret_cast<VT*>(K0)[vi] = pack(a);
}

// Local regions: zero the products of the seeds whose region leaves out block row I.
template <typename T, int SW>
__device__ __forceinline__ void region_mask(const uint32_t* __restrict__ mask, int W, int64_t I, int s0,
                                            T (&acc)[4][SW]) {
    const uint32_t bits = mask[I * W + s0 / 32] >> (s0 % 32);
#pragma unroll
    for (int i = 0; i < SW; ++i)
        if (!((bits >> i) & 1u))
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r][i] = (T)0;
}

// Block row Iu of Y = A X for the seeds s0 .. s0 + VEC - 1 (B >= VEC): the
// row's blocks are taken CH at a time, all indices, X vectors and values of a
// chunk requested before any is used; acc must start at zero.
template <typename T, int B, int CH>
__device__ __forceinline__ void spmm_row_vec(int64_t Iu, int s0, const int32_t* __restrict__ brp,
                                             const int32_t* __restrict__ bcol, const T* __restrict__ bval,
                                             const typename Vec16<T>::type* __restrict__ Xv,
                                             T (&acc)[4][SeedMap<T, B>::SW], bool far = false) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW;
    using VT = typename Vec16<T>::type;
    const int lo = brp[Iu], hi = far ? lo : brp[Iu + 1];   // far: a row where the product is exactly zero
    for (int b0 = lo; b0 < hi; b0 += CH) {
        int blk[CH];
        int64_t J[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            blk[t] = b0 + t < hi ? b0 + t : hi - 1;   // repeats the last block; its sum is skipped
            J[t] = bcol[blk[t]];
        }
        T xv[CH][4][VEC];
#pragma unroll
        for (int t = 0; t < CH; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) unpack(Xv[((4 * J[t] + c) * B + s0) / VEC], xv[t][c]);
        T a[CH][16];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const VT* av = reinterpret_cast<const VT*>(bval + (int64_t)blk[t] * 16);
#pragma unroll
            for (int q = 0; q < 16 / VEC; ++q) {
                T u[VEC];
                unpack(av[q], u);
#pragma unroll
                for (int i = 0; i < VEC; ++i) a[t][q * VEC + i] = u[i];
            }
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            if (b0 + t < hi) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int i = 0; i < SW; ++i) {
                        T sacc = acc[r][i];
                        sacc = fma(a[t][r * 4 + 0], xv[t][0][i], sacc);
                        sacc = fma(a[t][r * 4 + 1], xv[t][1][i], sacc);
                        sacc = fma(a[t][r * 4 + 2], xv[t][2][i], sacc);
                        sacc = fma(a[t][r * 4 + 3], xv[t][3][i], sacc);
                        acc[r][i] = sacc;
                    }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Y = A X over B seed-interleaved vectors, A in BSR 4x4. Thread = (block row,
// seed group). The 16 block values are read once per thread and reused for
// SW seeds; X rows of the block column are 16-byte vector loads.
// Blocks of a row are taken CH at a time: the CH column indices, then all
// 4*CH X vectors and block values are requested before any is used, so one
// memory latency covers CH blocks. When a wavefront holds one block row
// (P = 64) the row index is made wavefront-uniform, so indices and block
// values come through scalar loads.
// NDOT >= 1: also emit per-workgroup FP64 partial sums of X.Y per seed (the
// S-norm w^T S w of a residual when A = S); NDOT = 2 adds X.X. Partials are
// laid out part[wg][d][b].
template <typename T, int B, int NDOT>
__global__ __launch_bounds__(WG) void k_spmm_bsr4(int64_t nbrow, const int32_t* __restrict__ brp,
                                                  const int32_t* __restrict__ bcol, const T* __restrict__ bval,
                                                  const T* __restrict__ X, T* __restrict__ Y,
                                                  double* __restrict__ part, const int32_t* __restrict__ tdist,
                                                  int lim, const uint32_t* __restrict__ mask, int W,
                                                  const int32_t* __restrict__ rdist, int64_t ntile, int64_t chunk) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    using VT = typename Vec16<T>::type;
    const int64_t bid = chunk > 0 ? xcd_chunk(blockIdx.x, chunk) : xcd_remap(blockIdx.x, gridDim.x);
    if (bid >= ntile) return;
    if (tdist != nullptr && tdist[bid] > lim) {   // a tile outside the support (B >= VEC: one tile per workgroup)
        if constexpr (NDOT > 0)
            for (int i = threadIdx.x; i < NDOT * B; i += WG) part[bid * NDOT * B + i] = 0.0;
        return;
    }
    const int64_t g = bid * WG + threadIdx.x;
    const int64_t I = g / P;
    const int grp = threadIdx.x % P;
    const int s0 = (B < VEC) ? 0 : grp * VEC;
    const VT* Xv = reinterpret_cast<const VT*>(X);
    T acc[4][SW];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < SW; ++i) acc[r][i] = (T)0;
    if constexpr (B >= VEC) {
        constexpr int CH = P == 64 ? 4 : 2;   // blocks in flight per row
        int64_t Iu = I;
        if constexpr (P == 64) Iu = __builtin_amdgcn_readfirstlane((int)I);   // one row per wavefront
        if (Iu < nbrow) {
            // rdist: block rows farther than lim hops get the zero they hold without a gather (their
            // neighbours may lie in tiles no sweep of this seed block has written)
            spmm_row_vec<T, B, CH>(Iu, s0, brp, bcol, bval, Xv, acc, rdist != nullptr && rdist[Iu] > lim);
            if (mask != nullptr) region_mask<T, SW>(mask, W, Iu, s0, acc);   // local regions
            // non-temporal: later kernels read Y; this one reuses X (neighbour rows) from L2
            VT* Yv = reinterpret_cast<VT*>(Y);
#pragma unroll
            for (int r = 0; r < 4; ++r) store_nt(Yv + ((4 * Iu + r) * B + s0) / VEC, acc[r]);
        }
    } else if (I < nbrow) {
        const int lo = brp[I], hi = brp[I + 1];
        for (int blk = lo; blk < hi; ++blk) {
            const int64_t J = bcol[blk];
            T a[16];
            const VT* av = reinterpret_cast<const VT*>(bval + (int64_t)blk * 16);
#pragma unroll
            for (int q = 0; q < 16 / VEC; ++q) {
                T t[VEC];
                unpack(av[q], t);
#pragma unroll
                for (int i = 0; i < VEC; ++i) a[q * VEC + i] = t[i];
            }
            // B < VEC: one vector holds VEC / B rows of all B seeds
            T xv[4][SW];
            T t[4 * B];
#pragma unroll
            for (int q = 0; q < 4 * B / VEC; ++q) {
                T u[VEC];
                unpack(Xv[(4 * J * B) / VEC + q], u);
#pragma unroll
                for (int i = 0; i < VEC; ++i) t[q * VEC + i] = u[i];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int i = 0; i < SW; ++i) xv[c][i] = t[c * B + i];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int i = 0; i < SW; ++i) {
                    T s = acc[r][i];
                    s = fma(a[r * 4 + 0], xv[0][i], s);
                    s = fma(a[r * 4 + 1], xv[1][i], s);
                    s = fma(a[r * 4 + 2], xv[2][i], s);
                    s = fma(a[r * 4 + 3], xv[3][i], s);
                    acc[r][i] = s;
                }
        }
        VT* Yv = reinterpret_cast<VT*>(Y);
#pragma unroll
        for (int q = 0; q < 4 * B / VEC; ++q) {
            T u[VEC];
#pragma unroll
            for (int i = 0; i < VEC; ++i) u[i] = acc[(q * VEC + i) / B][(q * VEC + i) % B];
            Yv[(4 * I * B) / VEC + q] = pack(u);
        }
    }
    if constexpr (NDOT > 0) {
        double d[NDOT][SW];
#pragma unroll
        for (int v = 0; v < NDOT; ++v)
#pragma unroll
            for (int i = 0; i < SW; ++i) d[v][i] = 0.0;
        if (I < nbrow) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T xr[SW];
                if constexpr (B >= VEC) {
                    unpack(Xv[((4 * I + r) * B + s0) / VEC], xr);
                } else {
#pragma unroll
                    for (int i = 0; i < SW; ++i) xr[i] = X[(4 * I + r) * B + s0 + i];
                }
#pragma unroll
                for (int i = 0; i < SW; ++i) {
                    const double xv = (double)xr[i];
                    d[0][i] += xv * (double)acc[r][i];
                    if constexpr (NDOT > 1) d[1][i] += xv * xv;
                }
            }
        }
        __shared__ double lds[SeedReduce<P, SW, NDOT>::LDS];
        wg_seed_reduce<P, SW, NDOT>(d, lds, [&](int v, int b, double s) { part[(bid * NDOT + v) * B + b] = s; });
    }
}

// Block row Iu of Y = H X and Z = S X for the seeds s0 .. s0 + VEC - 1,
// masked to the seeds' regions when mask != nullptr, stored (non-temporally
// when NTS: a whole-cell sweep, whose X rows are worth keeping in L2 rather
// than the results); the S-norm partials X.(S X) and X.X of the row are added
// to d (NDOT > 0).
template <typename T, int B, int NDOT, bool NTS>
__device__ __forceinline__ void spmm2_row(int64_t Iu, int s0, const int32_t* __restrict__ brp,
                                          const int32_t* __restrict__ bcol, const T* __restrict__ hval,
                                          const T* __restrict__ sval, const typename Vec16<T>::type* __restrict__ Xv,
                                          T* __restrict__ Y, T* __restrict__ Z, const uint32_t* __restrict__ mask,
                                          int W, double (&d)[NDOT > 0 ? NDOT : 1][SeedMap<T, B>::SW],
                                          bool far = false) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW;
    using VT = typename Vec16<T>::type;
    constexpr int CH = 2;   // blocks in flight per row (two value sets per block)
    T ah[4][SW], as[4][SW];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < SW; ++i) ah[r][i] = as[r][i] = (T)0;
    const int lo = brp[Iu], hi = far ? lo : brp[Iu + 1];   // far: both products are exactly zero on the row
    for (int b0 = lo; b0 < hi; b0 += CH) {
        int blk[CH];
        int64_t J[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            blk[t] = b0 + t < hi ? b0 + t : hi - 1;   // repeats the last block; its sum is skipped
            J[t] = bcol[blk[t]];
        }
        T xv[CH][4][VEC];
#pragma unroll
        for (int t = 0; t < CH; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) unpack(Xv[((4 * J[t] + c) * B + s0) / VEC], xv[t][c]);
        T hv[CH][16], sv[CH][16];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const VT* hp = reinterpret_cast<const VT*>(hval + (int64_t)blk[t] * 16);
            const VT* sp = reinterpret_cast<const VT*>(sval + (int64_t)blk[t] * 16);
#pragma unroll
            for (int q = 0; q < 16 / VEC; ++q) {
                T u[VEC], w[VEC];
                unpack(hp[q], u);
                unpack(sp[q], w);
#pragma unroll
                for (int i = 0; i < VEC; ++i) {
                    hv[t][q * VEC + i] = u[i];
                    sv[t][q * VEC + i] = w[i];
                }
            }
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            if (b0 + t < hi) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int i = 0; i < SW; ++i) {
                        T h = ah[r][i], z = as[r][i];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            h = fma(hv[t][r * 4 + c], xv[t][c][i], h);
                            z = fma(sv[t][r * 4 + c], xv[t][c][i], z);
                        }
                        ah[r][i] = h;
                        as[r][i] = z;
                    }
            }
        }
    }
    if (mask != nullptr) {
        region_mask<T, SW>(mask, W, Iu, s0, ah);
        region_mask<T, SW>(mask, W, Iu, s0, as);
    }
    VT* Yv = reinterpret_cast<VT*>(Y);
    VT* Zv = reinterpret_cast<VT*>(Z);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if constexpr (NTS) {
            store_nt(Yv + ((4 * Iu + r) * B + s0) / VEC, ah[r]);
            store_nt(Zv + ((4 * Iu + r) * B + s0) / VEC, as[r]);
        } else {
            Yv[((4 * Iu + r) * B + s0) / VEC] = pack(ah[r]);
            Zv[((4 * Iu + r) * B + s0) / VEC] = pack(as[r]);
        }
    }
    if constexpr (NDOT > 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T xr[SW];
            unpack(Xv[((4 * Iu + r) * B + s0) / VEC], xr);
#pragma unroll
            for (int i = 0; i < SW; ++i) {
                const double xd = (double)xr[i];
                d[0][i] += xd * (double)as[r][i];
                if constexpr (NDOT > 1) d[1][i] += xd * xd;
            }
        }
    }
}

// Y = H X and Z = S X in one pass over X, for S stored on H's block pattern
// (zero blocks where S has none); B >= VEC only. NDOT as in k_spmm_bsr4, with
// the products taken against Z: X.(S X) and X.X per seed. One row tile of
// WG / P block rows per workgroup; tiles with tdist > lim are skipped.
template <typename T, int B, int NDOT>
__global__ __launch_bounds__(WG) void k_spmm2_bsr4(int64_t nbrow, const int32_t* __restrict__ brp,
                                                   const int32_t* __restrict__ bcol, const T* __restrict__ hval,
                                                   const T* __restrict__ sval, const T* __restrict__ X,
                                                   T* __restrict__ Y, T* __restrict__ Z, double* __restrict__ part,
                                                   const int32_t* __restrict__ tdist, int lim,
                                                   const uint32_t* __restrict__ mask, int W,
                                                   const int32_t* __restrict__ rdist, int64_t ntile,
                                                   int64_t chunk) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    static_assert(B >= VEC, "dual product needs one seed group per lane");
    using VT = typename Vec16<T>::type;
    const int64_t bid = chunk > 0 ? xcd_chunk(blockIdx.x, chunk) : xcd_remap(blockIdx.x, gridDim.x);
    if (bid >= ntile) return;
    if (tdist != nullptr && tdist[bid] > lim) {   // a tile outside the support
        if constexpr (NDOT > 0)
            for (int i = threadIdx.x; i < NDOT * B; i += WG) part[bid * NDOT * B + i] = 0.0;
        return;
    }
    const int s0 = (threadIdx.x % P) * VEC;
    const VT* Xv = reinterpret_cast<const VT*>(X);
    double d[NDOT > 0 ? NDOT : 1][SW];
#pragma unroll
    for (int v = 0; v < (NDOT > 0 ? NDOT : 1); ++v)
#pragma unroll
        for (int i = 0; i < SW; ++i) d[v][i] = 0.0;
    int64_t Iu = (bid * WG + threadIdx.x) / P;
    if constexpr (P == 64) Iu = __builtin_amdgcn_readfirstlane((int)Iu);   // one row per wavefront
    if (Iu < nbrow)
        spmm2_row<T, B, NDOT, true>(Iu, s0, brp, bcol, hval, sval, Xv, Y, Z, mask, W, d,
                                    rdist != nullptr && rdist[Iu] > lim);
    if constexpr (NDOT > 0) {
        __shared__ double lds[SeedReduce<P, SW, NDOT>::LDS];
        wg_seed_reduce<P, SW, NDOT>(d, lds, [&](int v, int b, double sdot) { part[(bid * NDOT + v) * B + b] = sdot; });
    }
}

// The same product over the row tiles of a list (local regions): entries
// [0, cnt[lim]) in a grid-stride loop; partials per workgroup, part[wg][d][b].
template <typename T, int B, int NDOT>
__global__ __launch_bounds__(WG) void k_spmm2_list(int64_t nbrow, const int32_t* __restrict__ brp,
                                                   const int32_t* __restrict__ bcol, const T* __restrict__ hval,
                                                   const T* __restrict__ sval, const T* __restrict__ X,
                                                   T* __restrict__ Y, T* __restrict__ Z, double* __restrict__ part,
                                                   const int32_t* __restrict__ list, const int32_t* __restrict__ cnt,
                                                   int lim, const uint32_t* __restrict__ mask, int W) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    static_assert(B >= VEC, "dual product needs one seed group per lane");
    using VT = typename Vec16<T>::type;
    const int s0 = (threadIdx.x % P) * VEC;
    const VT* Xv = reinterpret_cast<const VT*>(X);
    double d[NDOT > 0 ? NDOT : 1][SW];
#pragma unroll
    for (int v = 0; v < (NDOT > 0 ? NDOT : 1); ++v)
#pragma unroll
        for (int i = 0; i < SW; ++i) d[v][i] = 0.0;
    const int64_t ce = cnt[lim];
    for (int64_t e = blockIdx.x; e < ce; e += gridDim.x) {
        int64_t Iu = ((int64_t)list[e] * WG + threadIdx.x) / P;
        if constexpr (P == 64) Iu = __builtin_amdgcn_readfirstlane((int)Iu);
        if (Iu < nbrow) spmm2_row<T, B, NDOT, false>(Iu, s0, brp, bcol, hval, sval, Xv, Y, Z, mask, W, d);
    }
    if constexpr (NDOT > 0) {
        __shared__ double lds[SeedReduce<P, SW, NDOT>::LDS];
        wg_seed_reduce<P, SW, NDOT>(d, lds, [&](int v, int b, double sdot) {
            part[((int64_t)blockIdx.x * NDOT + v) * B + b] = sdot;
        });
    }
}

// Y = A X on the row tiles of a list (local regions), no partials.
template <typename T, int B>
__global__ __launch_bounds__(WG) void k_spmm_list(int64_t nbrow, const int32_t* __restrict__ brp,
                                                  const int32_t* __restrict__ bcol, const T* __restrict__ bval,
                                                  const T* __restrict__ X, T* __restrict__ Y,
                                                  const int32_t* __restrict__ list, const int32_t* __restrict__ cnt,
                                                  int lim, const uint32_t* __restrict__ mask, int W) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    static_assert(B >= VEC, "one seed group per lane");
    using VT = typename Vec16<T>::type;
    constexpr int CH = P == 64 ? 4 : 2;
    const int s0 = (threadIdx.x % P) * VEC;
    const VT* Xv = reinterpret_cast<const VT*>(X);
    VT* Yv = reinterpret_cast<VT*>(Y);
    const int64_t ce = cnt[lim];
    for (int64_t e = blockIdx.x; e < ce; e += gridDim.x) {
        int64_t Iu = ((int64_t)list[e] * WG + threadIdx.x) / P;
        if constexpr (P == 64) Iu = __builtin_amdgcn_readfirstlane((int)Iu);
        if (Iu >= nbrow) continue;
        T acc[4][SW];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int i = 0; i < SW; ++i) acc[r][i] = (T)0;
        spmm_row_vec<T, B, CH>(Iu, s0, brp, bcol, bval, Xv, acc);
        if (mask != nullptr) region_mask<T, SW>(mask, W, Iu, s0, acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) Yv[((4 * Iu + r) * B + s0) / VEC] = pack(acc[r]);
    }
}

// Y = A X with A in CSR (patterns without 4x4 block structure). Thread = (row, seed group).
template <typename T, int B, int NDOT>
__global__ __launch_bounds__(WG) void k_spmm_csr(int64_t nrow, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col, const T* __restrict__ val,
                                                 const T* __restrict__ X, T* __restrict__ Y,
                                                 double* __restrict__ part) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    using VT = typename Vec16<T>::type;
    const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t g = bid * WG + threadIdx.x;
    const int64_t i0 = g / P;
    const int grp = threadIdx.x % P;
    const int s0 = (B < VEC) ? 0 : grp * VEC;
    T acc[SW];
#pragma unroll
    for (int i = 0; i < SW; ++i) acc[i] = (T)0;
    if (i0 < nrow) {
        for (int t = rp[i0]; t < rp[i0 + 1]; ++t) {
            const int64_t c = col[t];
            const T a = val[t];
            if constexpr (B >= VEC) {
                T u[VEC];
                unpack(reinterpret_cast<const VT*>(X)[(c * B + s0) / VEC], u);
#pragma unroll
                for (int i = 0; i < SW; ++i) acc[i] = fma(a, u[i], acc[i]);
            } else {
#pragma unroll
                for (int i = 0; i < SW; ++i) acc[i] = fma(a, X[c * B + i], acc[i]);
            }
        }
        if constexpr (B >= VEC) {
            reinterpret_cast<VT*>(Y)[(i0 * B + s0) / VEC] = pack(acc);
        } else {
#pragma unroll
            for (int i = 0; i < SW; ++i) Y[i0 * B + i] = acc[i];
        }
    }
    if constexpr (NDOT > 0) {
        double d[NDOT][SW];
#pragma unroll
        for (int i = 0; i < SW; ++i) {
            const double xv = (i0 < nrow) ? (double)X[i0 * B + s0 + i] : 0.0;
            d[0][i] = xv * (double)acc[i];
            if constexpr (NDOT > 1) d[1][i] = xv * xv;
        }
        __shared__ double lds[SeedReduce<P, SW, NDOT>::LDS];
        wg_seed_reduce<P, SW, NDOT>(d, lds, [&](int v, int b, double s) { part[(bid * NDOT + v) * B + b] = s; });
    }
}

// ---------------------------------------------------------------------------
// Projection pass of CGS: for the basis slabs k in this workgroup's range,
//   out[s][k][b] = sum over this chunk's rows of basis_s[k][row][b] * x[row][b]
// (s = 0: K, s = 1: S K). Partial sums per chunk go to part[chunk][s][k][b];
// a second kernel reduces over chunks in a fixed order. The chunk of x stays
// in registers and is reused for every slab.
template <typename T, int B, int NS, int Q, int KG>
__global__ __launch_bounds__(WG) void k_proj(const T* __restrict__ b0, const T* __restrict__ b1, int64_t slab,
                                             int nk, int kps, const T* __restrict__ x, int64_t nvec,
                                             double* __restrict__ part) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    using VT = typename Vec16<T>::type;
    const int tid = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    const int64_t vbase = chunk * (WG * Q) + tid;
    const int64_t slabv = slab / VEC;
    const VT* xv = reinterpret_cast<const VT*>(x);
    const VT* bv0 = reinterpret_cast<const VT*>(b0);
    const VT* bv1 = reinterpret_cast<const VT*>(b1);
    T xr[Q][VEC];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t vi = vbase + (int64_t)q * WG;
        if (vi < nvec) unpack(xv[vi], xr[q]);
        else {
#pragma unroll
            for (int i = 0; i < VEC; ++i) xr[q][i] = (T)0;
        }
    }
    const int k0 = blockIdx.y * kps;
    const int k1 = min(nk, k0 + kps);
    __shared__ T lds[SeedReduce<P, SW, NS * KG>::LDS];
    for (int kb = k0; kb < k1; kb += KG) {
        T raw[NS][KG][VEC];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int kk = 0; kk < KG; ++kk)
#pragma unroll
                for (int i = 0; i < VEC; ++i) raw[s][kk][i] = (T)0;
        // branch-free: slab indices past the range repeat the last slab (sums
        // never emitted); out-of-range vectors read vector 0 against x = 0
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            const int k = kb + kk < k1 ? kb + kk : k1 - 1;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t vi = vbase + (int64_t)q * WG;
                const int64_t vs = vi < nvec ? vi : 0;
                T a[VEC];
                unpack(bv0[(int64_t)k * slabv + vs], a);
#pragma unroll
                for (int i = 0; i < VEC; ++i) raw[0][kk][i] = fma(a[i], xr[q][i], raw[0][kk][i]);
                if constexpr (NS == 2) {
                    T c[VEC];
                    unpack(bv1[(int64_t)k * slabv + vs], c);
#pragma unroll
                    for (int i = 0; i < VEC; ++i) raw[1][kk][i] = fma(c[i], xr[q][i], raw[1][kk][i]);
                }
            }
        }
        T acc[NS * KG][SW];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) {
#pragma unroll
                for (int i = 0; i < SW; ++i) acc[s * KG + kk][i] = (T)0;
#pragma unroll
                for (int i = 0; i < VEC; ++i) acc[s * KG + kk][i % SW] += raw[s][kk][i];
            }
        wg_seed_reduce<P, SW, NS * KG>(acc, lds, [&](int v, int b, T sum) {
            const int s = v / KG, k = kb + v % KG;
            if (k < k1) part[((chunk * NS + s) * nk + k) * B + b] = (double)sum;
        });
    }
}

// ---------------------------------------------------------------------------
// Update pass of CGS: x[row][b] -= sum_k basis[k][row][b] * c[k][b].
template <typename T, int B, int Q>
__global__ __launch_bounds__(WG) void k_upd(const T* __restrict__ basis, int64_t slab, int nk,
                                            const double* __restrict__ c, T* __restrict__ x, int64_t nvec) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, P = SM::P;
    using VT = typename Vec16<T>::type;
    const int tid = threadIdx.x;
    const int64_t vbase = (int64_t)blockIdx.x * (WG * Q) + tid;
    const int64_t slabv = slab / VEC;
    const int sb = (B < VEC) ? 0 : (tid % P) * VEC;
    VT* xv = reinterpret_cast<VT*>(x);
    const VT* bv = reinterpret_cast<const VT*>(basis);
    T acc[Q][VEC];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t vi = vbase + (int64_t)q * WG;
        if (vi < nvec) unpack(xv[vi], acc[q]);
        else {
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc[q][i] = (T)0;
        }
    }
    int64_t vsq[Q];  // always-valid load indices (out-of-range lanes read vector 0, never stored)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t vi = vbase + (int64_t)q * WG;
        vsq[q] = vi < nvec ? vi : 0;
    }
    for (int k = 0; k < nk; ++k) {
        T cv[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) cv[i] = (T)c[(int64_t)k * B + ((B < VEC) ? (i % B) : (sb + i))];
        T a[Q][VEC];
#pragma unroll
        for (int q = 0; q < Q; ++q) unpack(bv[(int64_t)k * slabv + vsq[q]], a[q]);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc[q][i] = fma(-a[q][i], cv[i], acc[q][i]);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t vi = vbase + (int64_t)q * WG;
        if (vi < nvec) xv[vi] = pack(acc[q]);
    }
}

// ---------------------------------------------------------------------------
// Append u_{n+1} = w / beta and s_{n+1} = (S w) / beta (zero for seeds that
// stopped: breakdown, invalid seed or padding).
template <typename T, int B>
__global__ __launch_bounds__(WG) void k_append(const T* __restrict__ W, const T* __restrict__ Z,
                                               const double* __restrict__ beta, const int32_t* __restrict__ active,
                                               T* __restrict__ Kn, T* __restrict__ SKn, int64_t nvec) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, P = SM::P;
    using VT = typename Vec16<T>::type;
    const int64_t vi = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (vi >= nvec) return;
    const int sb = (B < VEC) ? 0 : (threadIdx.x % P) * VEC;
    T w[VEC], z[VEC];
    unpack(reinterpret_cast<const VT*>(W)[vi], w);
    unpack(reinterpret_cast<const VT*>(Z)[vi], z);
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
        const int b = (B < VEC) ? (i % B) : (sb + i);
        if (active[b]) {
            const T bt = (T)beta[b];
            w[i] = w[i] / bt;
            z[i] = z[i] / bt;
        } else {
            w[i] = (T)0;
            z[i] = (T)0;
        }
    }
    reinterpret_cast<VT*>(Kn)[vi] = pack(w);
    reinterpret_cast<VT*>(SKn)[vi] = pack(z);
}

// ---------------------------------------------------------------------------
// Delayed-reorthogonalization schedule (basis K only, no S K stored).
//
// Projection sweep: for NR right-hand sides r_0..r_{NR-1} (S u~, S y, y),
//   part[group][r][k][b] = sum over the group's rows of K[k][row][b] * r[row][b].
// Split over slabs: a workgroup owns KG consecutive slabs and `tiles` row
// tiles (WG*Q vectors each); its KG x NR accumulators stay in registers across
// all its tiles and are reduced across the workgroup once at the end, so one
// partial per (group, r, k, b) leaves the kernel. The slab splits of one row
// group are consecutive logical workgroups, which the XCD remapping places on
// one XCD: they stream the same right-hand-side tiles at about the same time,
// so those re-reads are served by that XCD's L2 rather than HBM.
template <typename T, int B, int NR, int Q, int KG, bool NT>
__global__ __launch_bounds__(WG) void k_projr(const T* __restrict__ basis, int64_t slab, int nk, int nks,
                                              const T* __restrict__ r0, const T* __restrict__ r1,
                                              const T* __restrict__ r2, int64_t nvec, int tiles,
                                              double* __restrict__ part) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    using VT = typename Vec16<T>::type;
    const int tid = threadIdx.x;
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t grp = L / nks;
    const int k0 = (int)(L % nks) * KG;
    const int nkl = min(KG, nk - k0);
    const int64_t slabv = slab / VEC;
    const VT* bv = reinterpret_cast<const VT*>(basis) + (int64_t)k0 * slabv;
    const VT* rv[3] = {reinterpret_cast<const VT*>(r0), reinterpret_cast<const VT*>(r1),
                       reinterpret_cast<const VT*>(r2)};
    T raw[NR][KG][VEC];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
#pragma unroll
            for (int i = 0; i < VEC; ++i) raw[r][kk][i] = (T)0;
    // Branch-free inner loop (a guarded load makes the compiler wait for each
    // load before the next): out-of-range vectors read vector 0 and contribute
    // zero; slab indices past the range repeat the last slab and their sums
    // are never emitted.
    int koff[KG];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) koff[kk] = kk < nkl ? kk : nkl - 1;
    for (int tile = 0; tile < tiles; ++tile) {
        const int64_t tbase = (grp * tiles + tile) * (int64_t)(WG * Q);
        if (tbase >= nvec) break;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t vi = tbase + (int64_t)q * WG + tid;
            const bool ok = vi < nvec;
            const int64_t vs = ok ? vi : 0;
            T x[NR][VEC];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                unpack(rv[r][vs], x[r]);
#pragma unroll
                for (int i = 0; i < VEC; ++i) x[r][i] = ok ? x[r][i] : (T)0;
            }
            T a[KG][VEC];
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) {
                if constexpr (NT) unpack_nt(bv + (int64_t)koff[kk] * slabv + vs, a[kk]);
                else unpack(bv[(int64_t)koff[kk] * slabv + vs], a[kk]);
            }
#pragma unroll
            for (int kk = 0; kk < KG; ++kk)
#pragma unroll
                for (int r = 0; r < NR; ++r)
#pragma unroll
                    for (int i = 0; i < VEC; ++i) raw[r][kk][i] = fma(a[kk][i], x[r][i], raw[r][kk][i]);
        }
    }
    T acc[NR * KG][SW];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
#pragma unroll
            for (int i = 0; i < SW; ++i) acc[r * KG + kk][i] = (T)0;
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc[r * KG + kk][i % SW] += raw[r][kk][i];
        }
    __shared__ T red_lds[SeedReduce<P, SW, NR * KG>::LDS];
    wg_seed_reduce<P, SW, NR * KG>(acc, red_lds, [&](int v, int b, T sum) {
        const int r = v / KG, kk = v % KG;
        if (kk < nkl) part[((grp * NR + r) * nk + (k0 + kk)) * B + b] = (double)sum;
    });
}

// The projection sweep restricted to the support of the block: the same
// products as k_projr, taken only over the tiles on which a slab of the
// workgroup's chunk can be nonzero. Workgroup w takes (group g, chunk ks) from
// the plan, the list entries [g Tg, min((g + 1) Tg, cnt[min(k0 + KG - 1, n)]))
// and slabs k0 .. k0 + KG - 1, and writes one partial per (r, slab, seed) to
// part[((w * NR + r) * KG + kk) * B + b]. A tile is 4 * WG vectors: 4 / Q
// passes of Q vectors per thread.
template <typename T, int B, int NR, int Q, int KG, bool NT>
__global__ __launch_bounds__(WG) void k_projr_sp(const T* __restrict__ basis, int64_t slab, int n,
                                                 const T* __restrict__ r0, const T* __restrict__ r1,
                                                 const T* __restrict__ r2, int64_t nvec,
                                                 const int32_t* __restrict__ list, const int32_t* __restrict__ cnt,
                                                 const int32_t* __restrict__ plan, int64_t grid,
                                                 double* __restrict__ part) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    constexpr int SUB = 4 / Q;
    static_assert(SUB * Q == 4, "a tile is 4 * WG vectors");
    using VT = typename Vec16<T>::type;
    const int tid = threadIdx.x;
    // The plan uses nact <= gridDim.x workgroups; they are spread evenly over the
    // XCDs, consecutive numbers (the chunks of one group) on the same XCD.
    const int64_t nact = plan[2];
    if ((int64_t)blockIdx.x >= nact) return;
    const int64_t w = xcd_remap(blockIdx.x, nact);
    const int32_t* tg = plan + 8 + 2 * grid;
    const int g = tg[w];
    if (g < 0) return;
    const int ks = tg[grid + w];
    const int Tg = plan[1];
    const int nk = n + 1;
    const int k0 = ks * KG;
    const int nkl = min(KG, nk - k0);
    const int64_t e0 = (int64_t)g * Tg;
    const int64_t ce = cnt[min(k0 + KG - 1, n)];
    const int64_t e1 = e0 + Tg < ce ? e0 + Tg : ce;
    const int64_t slabv = slab / VEC;
    const VT* bv = reinterpret_cast<const VT*>(basis) + (int64_t)k0 * slabv;
    const VT* rv[3] = {reinterpret_cast<const VT*>(r0), reinterpret_cast<const VT*>(r1),
                       reinterpret_cast<const VT*>(r2)};
    T raw[NR][KG][VEC];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
#pragma unroll
            for (int i = 0; i < VEC; ++i) raw[r][kk][i] = (T)0;
    // Slab k0 + kk can be nonzero only on the first cnt[k0 + kk] entries of the distance-sorted list. With
    // the basis streamed from HBM (NT), on the later entries of the chunk it reads slab k0 + nkl - 1 again
    // (whose lines are loaded in the same step: no further HBM traffic) and multiplies by +0, the value
    // those rows hold. Cached sweeps fit the last-level cache and read the chunk's slabs on all its entries.
    int64_t klim[KG];
    bool act[KG];
    int koff[KG];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
        klim[kk] = kk < nkl ? cnt[k0 + kk] : 0;
        act[kk] = true;
        koff[kk] = kk < nkl ? kk : nkl - 1;
    }
    // the next tile's index is fetched one tile ahead, so its loads need not wait for it
    int64_t t = e0 < e1 ? list[e0] : 0;
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t tn = e + 1 < e1 ? list[e + 1] : 0;
        if constexpr (NT) {
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) {
                act[kk] = e < klim[kk];
                koff[kk] = act[kk] ? kk : nkl - 1;
            }
        }
#pragma unroll
        for (int sub = 0; sub < SUB; ++sub) {
            const int64_t tbase = t * (int64_t)(4 * WG) + (int64_t)sub * (WG * Q);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t vi = tbase + (int64_t)q * WG + tid;
                const bool ok = vi < nvec;
                const int64_t vs = ok ? vi : 0;
                T x[NR][VEC];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    unpack(rv[r][vs], x[r]);
#pragma unroll
                    for (int i = 0; i < VEC; ++i) x[r][i] = ok ? x[r][i] : (T)0;
                }
                T a[KG][VEC];
#pragma unroll
                for (int kk = 0; kk < KG; ++kk) {
                    if constexpr (NT) unpack_nt(bv + (int64_t)koff[kk] * slabv + vs, a[kk]);
                    else unpack(bv[(int64_t)koff[kk] * slabv + vs], a[kk]);
                    if constexpr (NT) {
#pragma unroll
                        for (int i = 0; i < VEC; ++i) a[kk][i] = act[kk] ? a[kk][i] : (T)0;
                    }
                }
#pragma unroll
                for (int kk = 0; kk < KG; ++kk)
#pragma unroll
                    for (int r = 0; r < NR; ++r)
#pragma unroll
                        for (int i = 0; i < VEC; ++i) raw[r][kk][i] = fma(a[kk][i], x[r][i], raw[r][kk][i]);
            }
        }
        t = tn;
    }
    T acc[NR * KG][SW];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
#pragma unroll
            for (int i = 0; i < SW; ++i) acc[r * KG + kk][i] = (T)0;
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc[r * KG + kk][i % SW] += raw[r][kk][i];
        }
    __shared__ T red_lds[SeedReduce<P, SW, NR * KG>::LDS];
    wg_seed_reduce<P, SW, NR * KG>(acc, red_lds, [&](int v, int b, T sum) {
        const int r = v / KG, kk = v % KG;
        if (kk < nkl) part[((w * NR + r) * KG + kk) * B + b] = (double)sum;
    });
}

// Projection of every basis vector of a block onto one fixed vector v (rows,
// FP64): part[(g * nk + k) * B + b] = sum over the rows of chunk g of
// K[k][i][b] v[i]. Grid (groups, nk).
template <typename T, int B>
__global__ __launch_bounds__(WG) void k_es_pdot(const T* __restrict__ basis, int64_t slab, int64_t M,
                                                const double* __restrict__ v, int64_t nvec, int64_t chunk,
                                                double* __restrict__ part) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, SW = SM::SW, P = SM::P;
    using VT = typename Vec16<T>::type;
    const int g = blockIdx.x, k = blockIdx.y, nk = gridDim.y;
    const VT* bv = reinterpret_cast<const VT*>(basis) + (int64_t)k * (slab / VEC);
    double acc[1][SW];
#pragma unroll
    for (int i = 0; i < SW; ++i) acc[0][i] = 0.0;
    const int64_t v0 = (int64_t)g * chunk, v1 = v0 + chunk < nvec ? v0 + chunk : nvec;
    for (int64_t vi = v0 + threadIdx.x; vi < v1; vi += WG) {
        T a[VEC];
        unpack(bv[vi], a);
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const int64_t e = vi * VEC + i;   // element (row e / B, seed e % B)
            const int64_t row = e / B;
            const double x = row < M ? v[row] : 0.0;
            acc[0][i % SW] += (double)a[i] * x;
        }
    }
    __shared__ double lds[SeedReduce<P, SW, 1>::LDS];
    wg_seed_reduce<P, SW, 1>(acc, lds, [&](int, int b, double sum) { part[((int64_t)g * nk + k) * B + b] = sum; });
}

// Q vectors per thread at vbase, vbase + WG, ... (all < nvec), slabs from kst on (the slabs below kst are
// zero on these rows). The loads of one slab share one base address, so they go out at constant offsets.
// ACC64: the running sums u~ - sum K cA and y - sum K cB are kept in FP64 and rounded to the basis
// precision once, when stored (for an FP32 basis at large nu, where the FP32 rounding of these sums over
// hundreds of slabs dominates the form's error).
template <typename T, int B, int Q, bool WANT_W, bool NT, bool ACC64>
__device__ __forceinline__ void upd2_body(int64_t vbase, int kst, T* __restrict__ basis, int64_t slab, int n,
                                          const T* __restrict__ cA, const T* __restrict__ cB,
                                          const double* __restrict__ gam, const double* __restrict__ Fn,
                                          const T* __restrict__ y, T* __restrict__ wout) {
    using SM = SeedMap<T, B>;
    constexpr int VEC = SM::VEC, P = SM::P;
    using VT = typename Vec16<T>::type;
    using AT = typename std::conditional<ACC64, double, T>::type;
    const int tid = threadIdx.x;
    const int64_t slabv = slab / VEC;
    const int sb = (B < VEC) ? 0 : (tid % P) * VEC;
    VT* bv = reinterpret_cast<VT*>(basis) + vbase;
    const VT* yv = reinterpret_cast<const VT*>(y) + vbase;
    AT au[Q][VEC], aw[Q][VEC];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T t0[VEC], t1[VEC];
        unpack(bv[(int64_t)n * slabv + q * WG], t0);
        if constexpr (WANT_W) unpack(yv[q * WG], t1);
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            au[q][i] = (AT)t0[i];
            if constexpr (WANT_W) aw[q][i] = (AT)t1[i];
        }
    }
    auto coef = [&](int k, T (&ca)[VEC], T (&cb)[VEC]) {
        if constexpr (B >= VEC) {
            unpack(reinterpret_cast<const VT*>(cA + (int64_t)k * B + sb)[0], ca);
            if constexpr (WANT_W) unpack(reinterpret_cast<const VT*>(cB + (int64_t)k * B + sb)[0], cb);
        } else {
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
                ca[i] = cA[(int64_t)k * B + i % B];
                if constexpr (WANT_W) cb[i] = cB[(int64_t)k * B + i % B];
            }
        }
    };
    auto step = [&](int q, const T (&a)[VEC], const T (&ca)[VEC], const T (&cb)[VEC]) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            au[q][i] = fma(-(AT)a[i], (AT)ca[i], au[q][i]);
            if constexpr (WANT_W) aw[q][i] = fma(-(AT)a[i], (AT)cb[i], aw[q][i]);
        }
    };
    if constexpr (NT && ACC64) {
        // Streaming from HBM with FP64 sums: the next vector's load is issued before this one's sums, so the
        // longer FP64 arithmetic runs under a load in flight (one load at a time left it exposed: 5.5 against
        // 6.1 TB/s on the 131072-row workload; with FP32 sums the same look-ahead was slower, 5.6 against 6.2)
        T an[VEC];
        if (kst < n) unpack_nt(bv + (int64_t)kst * slabv, an);
        for (int k = kst; k < n; ++k) {
            T ca[VEC], cb[VEC];
            coef(k, ca, cb);
            const VT* bk = bv + (int64_t)k * slabv;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                T a[VEC];
#pragma unroll
                for (int i = 0; i < VEC; ++i) a[i] = an[i];
                if (q + 1 < Q) unpack_nt(bk + (q + 1) * WG, an);
                else if (k + 1 < n) unpack_nt(bk + slabv, an);
                step(q, a, ca, cb);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        for (int k = kst; k < n; ++k) {
            T ca[VEC], cb[VEC];
            coef(k, ca, cb);
            // NT: the slabs swept exceed the last-level cache and are read once per sweep, so non-temporal
            // loads keep them from displacing reused lines; a smaller basis stays cached from one sweep to the
            // next
            const VT* bk = bv + (int64_t)k * slabv;
            if constexpr (NT) {
                // Streaming from HBM: one vector at a time, each load used before the next is issued (the
                // scheduling barrier keeps the compiler from hoisting them). Four loads in flight per wave
                // made this sweep 20 % slower (5.4 against 6.5 TB/s on the 131072-row workload).
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    T a[VEC];
                    unpack_nt(bk + q * WG, a);
                    step(q, a, ca, cb);
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                // cached slabs (a basis within the last-level cache, local regions): all loads in flight
                T a[Q][VEC];
#pragma unroll
                for (int q = 0; q < Q; ++q) unpack(bk[q * WG], a[q]);
#pragma unroll
                for (int q = 0; q < Q; ++q) step(q, a[q], ca, cb);
            }
        }
    }
    // 1 / gamma in FP64, rounded once: a multiply per element instead of a division, whose expansion held
    // registers enough to lower the sweep's occupancy
    AT rg[VEC], fn[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
        const int b = (B < VEC) ? (i % B) : (sb + i);
        rg[i] = (AT)(1.0 / gam[b]);
        fn[i] = (AT)Fn[b];
    }
    VT* wv = reinterpret_cast<VT*>(wout) + vbase;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T ou[VEC], ow[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            au[q][i] = au[q][i] * rg[i];
            if constexpr (WANT_W) aw[q][i] = (aw[q][i] - au[q][i] * fn[i]) * rg[i];
            ou[i] = (T)au[q][i];
            ow[i] = (T)aw[q][i];
        }
        if constexpr (NT) {   // a sweep beyond the last-level cache: the results too bypass it
            store_nt(bv + (int64_t)n * slabv + q * WG, ou);
            if constexpr (WANT_W) store_nt(wv + q * WG, ow);
        } else {
            bv[(int64_t)n * slabv + q * WG] = pack(ou);
            if constexpr (WANT_W) wv[q * WG] = pack(ow);
        }
    }
}

// One chunk of WG * Q vectors starting at v0, slabs from kst on. A whole chunk runs the branch-free body;
// the one chunk that reaches past nvec runs it vector by vector, for the lanes still inside.
template <typename T, int B, int Q, bool WANT_W, bool NT, bool ACC64>
__device__ __forceinline__ void upd2_chunk(int64_t v0, int kst, T* __restrict__ basis, int64_t slab, int n,
                                           const T* __restrict__ cA, const T* __restrict__ cB,
                                           const double* __restrict__ gam, const double* __restrict__ Fn,
                                           const T* __restrict__ y, T* __restrict__ wout, int64_t nvec) {
    const int64_t vbase = v0 + threadIdx.x;
    if (v0 + (int64_t)Q * WG <= nvec) {
        upd2_body<T, B, Q, WANT_W, NT, ACC64>(vbase, kst, basis, slab, n, cA, cB, gam, Fn, y, wout);
    } else {
        for (int q = 0; q < Q; ++q)
            if (vbase + (int64_t)q * WG < nvec)
                upd2_body<T, B, 1, WANT_W, NT, ACC64>(vbase + (int64_t)q * WG, kst, basis, slab, n, cA, cB, gam, Fn,
                                                      y, wout);
    }
}

// Dual update of the delayed schedule, one pass over slabs 0..n-1:
//   u_n = (u~ - sum_k K_k cA_k) / gamma       (second Gram-Schmidt pass of u~)
//   w'  = (y  - sum_k K_k cB_k - u_n F_n) / gamma   (first pass of y = H u~)
// u~ is slab n and is overwritten by u_n; w' goes to wout (WANT_W), the next
// slab, unnormalized. The slab may hold u~ times a per-seed scale s and y
// times the same s: the caller passes s cA, s cB, s F_n and s gamma.
// The coefficients are [k][B] in the basis precision: one 16-byte load per
// lane and slab for each of cA, cB when B >= VEC. One chunk of WG * Q
// vectors per workgroup; NT: non-temporal slab loads.
template <typename T, int B, int Q, bool WANT_W, bool NT, bool ACC64>
__global__ __launch_bounds__(WG) void k_upd2(T* __restrict__ basis, int64_t slab, int n, const T* __restrict__ cA,
                                             const T* __restrict__ cB, const double* __restrict__ gam,
                                             const double* __restrict__ Fn, const T* __restrict__ y,
                                             T* __restrict__ wout, int64_t nvec) {
    const int64_t v0 = (int64_t)blockIdx.x * (WG * Q);
    const int kst = 0;
    upd2_chunk<T, B, Q, WANT_W, NT, ACC64>(v0, kst, basis, slab, n, cA, cB, gam, Fn, y, wout, nvec);
}

// The same update over the row tiles of the support list, sorted by distance
// from the block's seeds: entries [0, cnt[lim]) in a grid-stride loop, one
// tile of 4 * WG vectors per step, its slab loop starting at the tile's
// distance Dl. Workgroups that run together take neighbouring entries, so they
// start at the same slab and stream the same slabs at the same time (tiles
// taken in row order start at scattered slabs, and the sweep then runs ~20 %
// slower). NT: non-temporal slab loads.
// Entries [cnt[lim], cnt[limz]) (WANT_W): the tiles just beyond w''s support
// get zeros in wout, so that the sweeps that read slab n + 1 a few hops past
// its support find the zeros it has there (slabs are not cleared per block).
// STRIDE = false: one entry per workgroup (the grid covers every tile); a grid-stride loop held registers
// enough to lower the sweep's occupancy.
template <typename T, int B, bool WANT_W, bool NT, bool STRIDE, bool ACC64>
__global__ __launch_bounds__(WG) void k_upd2_list(T* __restrict__ basis, int64_t slab, int n,
                                                  const T* __restrict__ cA, const T* __restrict__ cB,
                                                  const double* __restrict__ gam, const double* __restrict__ Fn,
                                                  const T* __restrict__ y, T* __restrict__ wout, int64_t nvec,
                                                  const int32_t* __restrict__ list, const int32_t* __restrict__ Dl,
                                                  const int32_t* __restrict__ cnt, int lim, int limz) {
    using VT = typename Vec16<T>::type;
    const int64_t ce = cnt[lim];
    const int64_t cz = WANT_W && limz > lim ? cnt[limz] : ce;
    for (int64_t e = blockIdx.x; e < cz; e += STRIDE ? (int64_t)gridDim.x : cz) {
        const int64_t t = list[e];
        if (e < ce) {
            upd2_chunk<T, B, 4, WANT_W, NT, ACC64>(t * (4 * WG), min(Dl[e], n), basis, slab, n, cA, cB, gam, Fn, y,
                                                   wout, nvec);
        } else if constexpr (WANT_W) {
            T z[Vec16<T>::n];
#pragma unroll
            for (int i = 0; i < Vec16<T>::n; ++i) z[i] = (T)0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t vi = t * (4 * WG) + (int64_t)q * WG + threadIdx.x;
                if (vi < nvec) reinterpret_cast<VT*>(wout)[vi] = pack(z);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers: dispatch the runtime block size B to the compiled instance.
#define MAR_DISPATCH_B(B, ...)                                   \
    switch (B) {                                                 \
        case 1: { constexpr int BB = 1; __VA_ARGS__; } break;    \
        case 2: { constexpr int BB = 2; __VA_ARGS__; } break;    \
        case 4: { constexpr int BB = 4; __VA_ARGS__; } break;    \
        case 8: { constexpr int BB = 8; __VA_ARGS__; } break;    \
        case 16: { constexpr int BB = 16; __VA_ARGS__; } break;  \
        case 32: { constexpr int BB = 32; __VA_ARGS__; } break;  \
        case 64: { constexpr int BB = 64; __VA_ARGS__; } break;  \
        case 128: { constexpr int BB = 128; __VA_ARGS__; } break;\
        default: MAR_DISPATCH_BIG(__VA_ARGS__);                  \
    }

template <>
LaunchInfo launch_init<MAR_T>(int B, int64_t Mp, int64_t M, const int32_t* seeds, int nseeds, const double* diagS,
                              int nu, MAR_T* K0, int32_t* active, int32_t* nu_eff, double* uu, hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    const int64_t nvec = Mp * B / VEC;
    const int64_t wgs = (std::max<int64_t>(nvec, B) + WG - 1) / WG;
    MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_init<MAR_T, BB>), dim3(wgs), dim3(WG), 0, s, Mp, M, seeds, nseeds,
                                         diagS, nu, K0, active, nu_eff, uu));
    LaunchInfo li;
    li.wgs = wgs;
    li.bytes = (double)Mp * B * sizeof(MAR_T);
    return li;
}

template <>
LaunchInfo launch_spmm<MAR_T>(int B, const DevMat& A, const MAR_T* X, MAR_T* Y, double* part, int ndot,
                              int64_t part_cap, hipStream_t s, const int32_t* tdist, int lim, const uint32_t* mask,
                              int W, const int32_t* rdist) {
    constexpr int VEC = Vec16<MAR_T>::n;
    const int P = B < VEC ? 1 : B / VEC;
    const int64_t wgs = (A.n * P + WG - 1) / WG;
    if ((ndot > 0 && wgs * ndot * B > part_cap) ||
        ((tdist != nullptr || mask != nullptr || rdist != nullptr) && (!A.bsr || B < VEC))) {
        LaunchInfo bad;
        bad.wgs = -1;
        return bad;
    }
    const MAR_T* val = std::is_same<MAR_T, float>::value ? (const MAR_T*)A.v32 : (const MAR_T*)A.v64;
#define MAR_SPMM_LAUNCH(KERNEL, ND) \
    MAR_DISPATCH_B(B, hipLaunchKernelGGL((KERNEL<MAR_T, BB, ND>), dim3(wgs), dim3(WG), 0, s, A.n, A.ptr, A.idx, val, X, Y, part))
    // whole-cell products: chunk-interleaved tile order when the pattern's far neighbours are far enough
    const int64_t chunk = A.bsr ? spmm_chunk(A.span, WG / P) : 0;
    const int64_t grid = chunk > 0 ? (wgs + 8 * chunk - 1) / (8 * chunk) * (8 * chunk) : wgs;
#define MAR_SPMM_BSR(ND) \
    MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_spmm_bsr4<MAR_T, BB, ND>), dim3((unsigned)grid), dim3(WG), 0, s, A.n, A.ptr, A.idx, val, X, Y, part, tdist, lim, mask, W, rdist, wgs, chunk))
    if (A.bsr) {
        if (ndot == 2) { MAR_SPMM_BSR(2); }
        else if (ndot == 1) { MAR_SPMM_BSR(1); }
        else { MAR_SPMM_BSR(0); }
#undef MAR_SPMM_BSR
    } else {
        if (ndot == 2) { MAR_SPMM_LAUNCH(k_spmm_csr, 2); }
        else if (ndot == 1) { MAR_SPMM_LAUNCH(k_spmm_csr, 1); }
        else { MAR_SPMM_LAUNCH(k_spmm_csr, 0); }
    }
#undef MAR_SPMM_LAUNCH
    const int64_t rows = A.bsr ? 4 * A.n : A.n;
    LaunchInfo li;
    li.wgs = wgs;
    li.bytes = A.bytes_per_pass(sizeof(MAR_T)) + 2.0 * (double)rows * B * sizeof(MAR_T);
    li.flops = 2.0 * (double)A.nnz * (A.bsr ? 16.0 : 1.0) * B;
    return li;
}

template <>
LaunchInfo launch_spmm2<MAR_T>(int B, const DevMat& H, const DevMat& SH, const MAR_T* X, MAR_T* Y, MAR_T* Z,
                               double* part, int ndot, int64_t part_cap, hipStream_t s, const int32_t* tdist,
                               int lim, const uint32_t* mask, int W, const int32_t* rdist) {
    constexpr int VEC = Vec16<MAR_T>::n;
    LaunchInfo li;
    if (!H.bsr || B < VEC || SH.nnz != H.nnz) {
        li.wgs = -1;
        return li;
    }
    const int P = B / VEC;
    const int64_t wgs = (H.n * P + WG - 1) / WG;
    if (ndot > 0 && wgs * ndot * B > part_cap) {
        li.wgs = -1;
        return li;
    }
    const bool f32 = std::is_same<MAR_T, float>::value;
    const MAR_T* hv = f32 ? (const MAR_T*)H.v32 : (const MAR_T*)H.v64;
    const MAR_T* sv = f32 ? (const MAR_T*)SH.v32 : (const MAR_T*)SH.v64;
    const int64_t chunk = spmm_chunk(H.span, WG / P);
    const int64_t grid = chunk > 0 ? (wgs + 8 * chunk - 1) / (8 * chunk) * (8 * chunk) : wgs;
#define MAR_SPMM2(ND) \
    MAR_DISPATCH_B(B, if constexpr (BB >= VEC) hipLaunchKernelGGL((k_spmm2_bsr4<MAR_T, BB, ND>), dim3((unsigned)grid), dim3(WG), 0, s, H.n, H.ptr, H.idx, hv, sv, X, Y, Z, part, tdist, lim, mask, W, rdist, wgs, chunk))
    if (ndot == 2) { MAR_SPMM2(2); }
    else if (ndot == 1) { MAR_SPMM2(1); }
    else { MAR_SPMM2(0); }
#undef MAR_SPMM2
    li.wgs = wgs;
    li.bytes = (double)H.nnz * (2.0 * 16.0 * sizeof(MAR_T) + 4.0) + (double)(H.n + 1) * 4.0 +
               3.0 * (double)(4 * H.n) * B * sizeof(MAR_T);
    li.flops = 4.0 * (double)H.nnz * 16.0 * B;
    return li;
}

template <>
LaunchInfo launch_spmm2_list<MAR_T>(int B, const DevMat& H, const DevMat& SH, const MAR_T* X, MAR_T* Y, MAR_T* Z,
                                    double* part, int ndot, int64_t part_cap, const int32_t* list, const int32_t* cnt,
                                    int lim, const uint32_t* mask, int W, int64_t grid, hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    LaunchInfo li;
    if (!H.bsr || B < VEC || SH.nnz != H.nnz || (ndot > 0 && grid * ndot * B > part_cap)) {
        li.wgs = -1;
        return li;
    }
    const bool f32 = std::is_same<MAR_T, float>::value;
    const MAR_T* hv = f32 ? (const MAR_T*)H.v32 : (const MAR_T*)H.v64;
    const MAR_T* sv = f32 ? (const MAR_T*)SH.v32 : (const MAR_T*)SH.v64;
#define MAR_SPMM2L(ND) \
    MAR_DISPATCH_B(B, if constexpr (BB >= VEC) hipLaunchKernelGGL((k_spmm2_list<MAR_T, BB, ND>), dim3((unsigned)grid), dim3(WG), 0, s, H.n, H.ptr, H.idx, hv, sv, X, Y, Z, part, list, cnt, lim, mask, W))
    if (ndot == 2) { MAR_SPMM2L(2); }
    else if (ndot == 1) { MAR_SPMM2L(1); }
    else { MAR_SPMM2L(0); }
#undef MAR_SPMM2L
    li.wgs = grid;
    li.bytes = (double)H.nnz * (2.0 * 16.0 * sizeof(MAR_T) + 4.0) + (double)(H.n + 1) * 4.0 +
               3.0 * (double)(4 * H.n) * B * sizeof(MAR_T);
    li.flops = 4.0 * (double)H.nnz * 16.0 * B;
    return li;
}

template <>
LaunchInfo launch_spmm_list<MAR_T>(int B, const DevMat& A, const MAR_T* X, MAR_T* Y, const int32_t* list,
                                   const int32_t* cnt, int lim, const uint32_t* mask, int W, int64_t grid,
                                   hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    LaunchInfo li;
    if (!A.bsr || B < VEC) {
        li.wgs = -1;
        return li;
    }
    const MAR_T* val = std::is_same<MAR_T, float>::value ? (const MAR_T*)A.v32 : (const MAR_T*)A.v64;
    MAR_DISPATCH_B(B, if constexpr (BB >= VEC) hipLaunchKernelGGL((k_spmm_list<MAR_T, BB>), dim3((unsigned)grid), dim3(WG), 0, s, A.n, A.ptr, A.idx, val, X, Y, list, cnt, lim, mask, W))
    li.wgs = grid;
    li.bytes = A.bytes_per_pass(sizeof(MAR_T)) + 2.0 * (double)(4 * A.n) * B * sizeof(MAR_T);
    li.flops = 2.0 * (double)A.nnz * 16.0 * B;
    return li;
}

template <>
LaunchInfo launch_proj<MAR_T>(int B, int ns, const MAR_T* b0, const MAR_T* b1, int64_t M, int64_t stride, int nk,
                              const MAR_T* x, double* part, int64_t part_cap, int64_t* nchunks, hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    const int64_t nvec = M * B / VEC;
    const int64_t chunks = (nvec + WG * PROJ_Q - 1) / (WG * PROJ_Q);
    // split the slabs over more workgroups when the chunks alone cannot fill the GPU
    const int64_t want = 2048;
    int64_t nks = std::max<int64_t>(1, (want + chunks - 1) / chunks);
    nks = std::min<int64_t>(nks, (nk + PROJ_KG - 1) / PROJ_KG);
    int kps = (int)((nk + nks - 1) / nks);
    kps = ((kps + PROJ_KG - 1) / PROJ_KG) * PROJ_KG;
    nks = (nk + kps - 1) / kps;
    const int64_t slab = stride;
    if (chunks * ns * nk * B > part_cap) {
        LaunchInfo bad;
        bad.wgs = -1;
        return bad;
    }
    dim3 grid((unsigned)chunks, (unsigned)nks);
    if (ns == 2) {
        MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_proj<MAR_T, BB, 2, PROJ_Q, PROJ_KG>), grid, dim3(WG), 0, s, b0, b1,
                                             slab, nk, kps, x, nvec, part));
    } else {
        MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_proj<MAR_T, BB, 1, PROJ_Q, PROJ_KG>), grid, dim3(WG), 0, s, b0, b1,
                                             slab, nk, kps, x, nvec, part));
    }
    *nchunks = chunks;
    LaunchInfo li;
    li.wgs = chunks * nks;
    li.bytes = ((double)ns * nk + 1.0) * (double)(M * B) * sizeof(MAR_T);
    li.flops = 2.0 * ns * nk * (double)(M * B);
    return li;
}

template <>
LaunchInfo launch_upd<MAR_T>(int B, const MAR_T* basis, int64_t M, int64_t stride, int nk, const double* c,
                             MAR_T* x, hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    const int64_t nvec = M * B / VEC;
    const int64_t slab = stride;
    const bool big = nvec >= (int64_t)WG * 4 * 1024;
    LaunchInfo li;
    if (big) {
        const int64_t wgs = (nvec + WG * 4 - 1) / (WG * 4);
        MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_upd<MAR_T, BB, 4>), dim3(wgs), dim3(WG), 0, s, basis, slab, nk, c,
                                             x, nvec));
        li.wgs = wgs;
    } else {
        const int64_t wgs = (nvec + WG - 1) / WG;
        MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_upd<MAR_T, BB, 1>), dim3(wgs), dim3(WG), 0, s, basis, slab, nk, c,
                                             x, nvec));
        li.wgs = wgs;
    }
    li.bytes = ((double)nk + 2.0) * (double)(M * B) * sizeof(MAR_T);
    li.flops = 2.0 * nk * (double)(M * B);
    return li;
}

template <>
LaunchInfo launch_append<MAR_T>(int B, int64_t M, const MAR_T* W, const MAR_T* Z, const double* beta,
                                const int32_t* active, MAR_T* Kn, MAR_T* SKn, hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    const int64_t nvec = M * B / VEC;
    const int64_t wgs = (nvec + WG - 1) / WG;
    MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_append<MAR_T, BB>), dim3(wgs), dim3(WG), 0, s, W, Z, beta, active, Kn,
                                         SKn, nvec));
    LaunchInfo li;
    li.wgs = wgs;
    li.bytes = 4.0 * (double)M * B * sizeof(MAR_T);
    return li;
}

template <>
LaunchInfo launch_projr<MAR_T>(int B, const MAR_T* basis, int64_t M, int64_t stride, int nk, const MAR_T* r0,
                               const MAR_T* r1, const MAR_T* r2, double* part, int64_t part_cap, int64_t* ngroups,
                               int64_t target_wgs, int variant, hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    constexpr int NR = 3;
    const int64_t nvec = M * B / VEC;
    const ProjrGeom gm = projr_geometry(nvec, nk, variant, target_wgs);
    const int nks = gm.nks;
    const int64_t tiles = gm.tiles, groups = gm.groups;
    const int64_t wgs = groups * nks;
    if (groups * NR * nk * B > part_cap) {
        LaunchInfo bad;
        bad.wgs = -1;
        return bad;
    }
#define MAR_PROJR(QV, KGV, NTV) \
    MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_projr<MAR_T, BB, NR, QV, KGV, NTV>), dim3((unsigned)wgs), dim3(WG), 0, s, basis, stride, nk, nks, r0, r1, r2, nvec, (int)tiles, part))
    if (variant == 1) { MAR_PROJR(PROJR_Q, 8, false); }
    else if (variant == 2) { MAR_PROJR(PROJR_Q, 4, true); }
    else if (variant == 3) { MAR_PROJR(2, 4, false); }
    else if (variant == 4) { MAR_PROJR(2, 8, false); }
    else if (variant == 5) { MAR_PROJR(PROJR_Q, 6, false); }
    else if (variant == 6) { MAR_PROJR(2, 6, false); }
    else if (variant == 7) { MAR_PROJR(PROJR_Q, 8, true); }
    else { MAR_PROJR(PROJR_Q, 4, false); }
#undef MAR_PROJR
    *ngroups = groups;
    LaunchInfo li;
    li.wgs = wgs;
    li.bytes = ((double)nk + NR) * (double)(M * B) * sizeof(MAR_T);
    li.flops = 2.0 * NR * nk * (double)(M * B);
    return li;
}

template <>
int projr_blocks_per_cu<MAR_T>(int B, int variant) {
    int nb = 0;
#define MAR_OCC(QV, KGV, NTV) \
    MAR_DISPATCH_B(B, (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_projr<MAR_T, BB, 3, QV, KGV, NTV>), WG, 0))
    if (variant == 1) { MAR_OCC(PROJR_Q, 8, false); }
    else if (variant == 2) { MAR_OCC(PROJR_Q, 4, true); }
    else if (variant == 3) { MAR_OCC(2, 4, false); }
    else if (variant == 4) { MAR_OCC(2, 8, false); }
    else if (variant == 5) { MAR_OCC(PROJR_Q, 6, false); }
    else if (variant == 6) { MAR_OCC(2, 6, false); }
    else if (variant == 7) { MAR_OCC(PROJR_Q, 8, true); }
    else { MAR_OCC(PROJR_Q, 4, false); }
#undef MAR_OCC
    return nb > 0 ? nb : 1;
}

template <>
LaunchInfo launch_projr_sp<MAR_T>(int B, const MAR_T* basis, int64_t M, int64_t stride, int n, const MAR_T* r0,
                                  const MAR_T* r1, const MAR_T* r2, const int32_t* list, const int32_t* cnt,
                                  const int32_t* plan, int64_t grid, double* part, int64_t part_cap, int variant,
                                  hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    constexpr int NR = 3;
    const int64_t nvec = M * B / VEC;
    const int kg = projr_kg(variant);
    const int64_t nks = (n + 1 + kg - 1) / kg;
    // one round of the device: the plan uses at most max(G, chunks) workgroups (grid = G + chunks)
    const int64_t wgs = std::max(grid - nks, nks);
    if (B < VEC || grid * NR * kg * B > part_cap) {
        LaunchInfo bad;
        bad.wgs = -1;
        return bad;
    }
#define MAR_PROJR_SP(QV, KGV, NTV) \
    MAR_DISPATCH_B(B, if constexpr (BB >= VEC) hipLaunchKernelGGL((k_projr_sp<MAR_T, BB, NR, QV, KGV, NTV>), dim3((unsigned)wgs), dim3(WG), 0, s, basis, stride, n, r0, r1, r2, nvec, list, cnt, plan, grid, part))
    if (variant == 1) { MAR_PROJR_SP(PROJR_Q, 8, false); }
    else if (variant == 2) { MAR_PROJR_SP(PROJR_Q, 4, true); }
    else if (variant == 3) { MAR_PROJR_SP(2, 4, false); }
    else if (variant == 4) { MAR_PROJR_SP(2, 8, false); }
    else if (variant == 5) { MAR_PROJR_SP(PROJR_Q, 6, false); }
    else if (variant == 6) { MAR_PROJR_SP(2, 6, false); }
    else if (variant == 7) { MAR_PROJR_SP(PROJR_Q, 8, true); }
    else { MAR_PROJR_SP(PROJR_Q, 4, false); }
#undef MAR_PROJR_SP
    LaunchInfo li;
    li.wgs = wgs;
    // full-sweep figures; the profiler replaces them by the support-restricted ones
    li.bytes = ((double)(n + 1) + NR) * (double)(M * B) * sizeof(MAR_T);
    li.flops = 2.0 * NR * (n + 1) * (double)(M * B);
    return li;
}

template <>
LaunchInfo launch_es_pdot<MAR_T>(int B, const MAR_T* K, int64_t stride, int64_t M, int64_t Mp, int nu,
                                 const double* vref, double* part, int groups, hipStream_t s) {
    constexpr int VEC = Vec16<MAR_T>::n;
    const int64_t nvec = Mp * B / VEC;
    const int64_t chunk = ((nvec + groups - 1) / groups + WG - 1) / WG * WG;
    MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_es_pdot<MAR_T, BB>), dim3(groups, nu), dim3(WG), 0, s, K, stride, M, vref, nvec, chunk, part))
    LaunchInfo li;
    li.wgs = (int64_t)groups * nu;
    li.bytes = (double)nu * Mp * B * sizeof(MAR_T) + (double)M * 8.0;
    li.flops = 2.0 * nu * (double)Mp * B;
    return li;
}

template <>
LaunchInfo launch_upd2_list<MAR_T>(int B, MAR_T* basis, int64_t M, int64_t stride, int n, const MAR_T* cA,
                                   const MAR_T* cB, const double* gam, const double* Fn, const MAR_T* y, MAR_T* wout,
                                   bool want_w, const int32_t* list, const int32_t* Dl, const int32_t* cnt, int lim,
                                   int limz, int64_t grid, bool nt, hipStream_t s, bool acc64) {
    constexpr int VEC = Vec16<MAR_T>::n;
    constexpr bool F32 = std::is_same<MAR_T, float>::value;
    const int64_t nvec = M * B / VEC;
    LaunchInfo li;
    if (B < VEC) {
        li.wgs = -1;
        return li;
    }
    // a grid of one workgroup per tile takes one entry each; a smaller grid loops over the entries
    const bool stride_loop = grid < (nvec + 4 * WG - 1) / (4 * WG);
#define MAR_UPD2L_(WW, NTT, SS, AA) \
    MAR_DISPATCH_B(B, if constexpr (BB >= VEC) hipLaunchKernelGGL((k_upd2_list<MAR_T, BB, WW, NTT, SS, AA>), dim3((unsigned)grid), dim3(WG), 0, s, basis, stride, n, cA, cB, gam, Fn, y, wout, nvec, list, Dl, cnt, lim, limz))
    // FP64 sums only for an FP32 basis (an FP64 basis sums in FP64 anyway)
#define MAR_UPD2L(WW, NTT, SS) \
    if (F32 && acc64) { MAR_UPD2L_(WW, NTT, SS, F32); } else { MAR_UPD2L_(WW, NTT, SS, false); }
    if (stride_loop) {   // local regions: few tiles, cached loads
        if (want_w) { MAR_UPD2L(true, false, true); } else { MAR_UPD2L(false, false, true); }
    } else if (nt) {
        if (want_w) { MAR_UPD2L(true, true, false); } else { MAR_UPD2L(false, true, false); }
    } else {
        if (want_w) { MAR_UPD2L(true, false, false); } else { MAR_UPD2L(false, false, false); }
    }
#undef MAR_UPD2L
#undef MAR_UPD2L_
    li.wgs = grid;
    const double slabs_read = (double)n + (want_w ? 2.0 : 1.0), slabs_written = want_w ? 2.0 : 1.0;
    li.bytes = (slabs_read + slabs_written) * (double)(M * B) * sizeof(MAR_T);
    li.flops = (want_w ? 4.0 : 2.0) * n * (double)(M * B);
    return li;
}

template <>
LaunchInfo launch_upd2<MAR_T>(int B, MAR_T* basis, int64_t M, int64_t stride, int n, const MAR_T* cA,
                              const MAR_T* cB, const double* gam, const double* Fn, const MAR_T* y, MAR_T* wout,
                              bool want_w, int upd_q, hipStream_t s, bool acc64) {
    constexpr int VEC = Vec16<MAR_T>::n;
    constexpr bool F32 = std::is_same<MAR_T, float>::value;
    const int64_t nvec = M * B / VEC;
    // vectors per thread: the requested depth when the grid still has >= 1024 workgroups
    int Q = upd_q == 2 || upd_q == 4 || upd_q == 8 ? upd_q : 4;
    while (Q > 1 && nvec < (int64_t)WG * Q * 1024) Q /= 2;
    const int64_t wgs = (nvec + WG * Q - 1) / (WG * Q);
    // non-temporal slab loads once the slabs swept are well beyond the 256 MB last-level cache (a smaller basis
    // is served from it sweep after sweep); the small-grid depths (Q < 4) always load through the caches
    const bool nt = (double)(n + 2) * (double)(M * B) * sizeof(MAR_T) > kNtSweepBytes;
#define MAR_UPD2_(QQ, WW, NTT, AA) \
    MAR_DISPATCH_B(B, hipLaunchKernelGGL((k_upd2<MAR_T, BB, QQ, WW, NTT, AA>), dim3(wgs), dim3(WG), 0, s, basis, stride, n, cA, cB, gam, Fn, y, wout, nvec))
#define MAR_UPD2(QQ, WW, NTT) \
    if (F32 && acc64) { MAR_UPD2_(QQ, WW, NTT, F32); } else { MAR_UPD2_(QQ, WW, NTT, false); }
#define MAR_UPD2W(QQ, NTT) \
    if (want_w) { MAR_UPD2(QQ, true, NTT); } else { MAR_UPD2(QQ, false, NTT); }
    if (Q == 8) { if (nt) { MAR_UPD2W(8, true) } else { MAR_UPD2W(8, false) } }
    else if (Q == 4) { if (nt) { MAR_UPD2W(4, true) } else { MAR_UPD2W(4, false) } }
    else if (Q == 2) { MAR_UPD2W(2, false) }
    else { MAR_UPD2W(1, false) }
#undef MAR_UPD2W
#undef MAR_UPD2
#undef MAR_UPD2_
    LaunchInfo li;
    li.wgs = wgs;
    const double slabs_read = (double)n + (want_w ? 2.0 : 1.0), slabs_written = want_w ? 2.0 : 1.0;
    li.bytes = (slabs_read + slabs_written) * (double)(M * B) * sizeof(MAR_T);
    li.flops = (want_w ? 4.0 : 2.0) * n * (double)(M * B);
    return li;
}

}  // namespace mar
