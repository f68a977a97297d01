// Device helpers shared by the streaming kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mar {

// 16-byte vector of T: one global_load/store_dwordx4 per lane.
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef double2 type; static constexpr int n = 2; };

__device__ __forceinline__ void unpack(const float4& v, float (&a)[4]) { a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w; }
__device__ __forceinline__ void unpack(const double2& v, double (&a)[2]) { a[0] = v.x; a[1] = v.y; }
__device__ __forceinline__ float4 pack(const float (&a)[4]) { return make_float4(a[0], a[1], a[2], a[3]); }
__device__ __forceinline__ double2 pack(const double (&a)[2]) { return make_double2(a[0], a[1]); }

// Non-temporal 16-byte loads (streamed data that should not displace reused lines in L2).
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef double nd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void unpack_nt(const float4* p, float (&a)[4]) {
    const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(p));
    a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
}
__device__ __forceinline__ void unpack_nt(const double2* p, double (&a)[2]) {
    const nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(p));
    a[0] = v.x; a[1] = v.y;
}

// Non-temporal 16-byte stores: results that only later kernels read, kept from displacing the lines
// that the storing kernel still reuses from L2.
__device__ __forceinline__ void store_nt(float4* p, const float (&a)[4]) {
    const nf4 v = {a[0], a[1], a[2], a[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<nf4*>(p));
}
__device__ __forceinline__ void store_nt(double2* p, const double (&a)[2]) {
    const nd2 v = {a[0], a[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<nd2*>(p));
}

// Seed-interleaved vectors: element e of an [M][B] array belongs to row e / B
// and seed e % B. A lane owns one 16-byte vector of VEC elements:
//   B >= VEC: the vector covers seeds (lane_vector_index % P) * VEC + [0, VEC),
//             P = B / VEC lanes share a row;
//   B <  VEC: the vector covers VEC / B rows of all B seeds; element i is seed i % B.
template <typename T, int B>
struct SeedMap {
    static constexpr int VEC = Vec16<T>::n;
    static constexpr int SW = B < VEC ? B : VEC;   // seeds per lane after folding
    static constexpr int P = B < VEC ? 1 : B / VEC; // lanes per row (distinct seed groups)
    static_assert(P <= 64, "B too large for one wavefront per row group");
};

// Map a hardware workgroup id to a logical one so that consecutive logical ids
// run on the same XCD (the dispatcher deals workgroups round-robin over 8 XCDs,
// each with its own L2). Bijective on [0, n).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t n) {
    constexpr int NX = 8;
    const int64_t per = n / NX, rem = n % NX;
    const int64_t x = bid % NX, local = bid / NX;
    return x * per + (x < rem ? x : rem) + local;
}

// Chunk-interleaved order: the dispatcher deals workgroup ids round-robin over the 8 XCDs, and XCD x takes
// the x-th chunk of each run of 8 chunks of `chunk` consecutive tiles, in order. When a run of 8 chunks
// spans the distance to a row's far neighbours (the next plane of cells of a lattice), those neighbours
// were read by the same XCD one chunk earlier instead of a whole contiguous range away. Bijective on
// [0, 8 * chunk * k); ids past the real tiles are skipped by the caller.
__device__ __forceinline__ int64_t xcd_chunk(int64_t bid, int64_t chunk) {
    constexpr int NX = 8;
    const int64_t x = bid % NX, l = bid / NX;
    return ((l / chunk) * NX + x) * chunk + l % chunk;
}

// Workgroup reduction of per-seed partial sums (fixed order, deterministic).
// Thread t holds vals[v][i] for seed (t % P) * SW + i. For every v and every
// seed b in [0, P*SW) the sum over the workgroup's 256 threads is passed to
// emit(v, b, sum) by exactly one thread (always the same thread for a given
// (v, b)). Values cross waves through LDS in chunks of SeedReduce::NVC values,
// so the exchange buffer holds SeedReduce::LDS elements whatever NV is.
template <int P, int SW, int NV>
struct SeedReduce {
    static constexpr int NVC_RAW = 768 / (P * SW);
    static constexpr int NVC = NVC_RAW < 1 ? 1 : (NVC_RAW > NV ? NV : NVC_RAW);
    static constexpr int LDS = 4 * NVC * P * SW;
};

template <int P, int SW, int NV, typename A, typename F>
__device__ __forceinline__ void wg_seed_reduce(A (&vals)[NV][SW], A* lds, F&& emit) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if constexpr (P < 64) {
#pragma unroll
        for (int off = P; off < 64; off <<= 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int i = 0; i < SW; ++i) vals[v][i] += __shfl_xor(vals[v][i], off);
        }
    }
    constexpr int NVC = SeedReduce<P, SW, NV>::NVC;
    constexpr int TOT = NVC * P * SW;
#pragma unroll
    for (int c0 = 0; c0 < NV; c0 += NVC) {
        if (lane < P) {
#pragma unroll
            for (int v = 0; v < NVC; ++v)
                if (c0 + v < NV) {
#pragma unroll
                    for (int i = 0; i < SW; ++i) lds[wave * TOT + (v * P + lane) * SW + i] = vals[c0 + v][i];
                }
        }
        __syncthreads();
        for (int o = threadIdx.x; o < TOT; o += 256) {
            const int v = c0 + o / (P * SW);
            if (v < NV) {
                A s = lds[o];
                s += lds[TOT + o];
                s += lds[2 * TOT + o];
                s += lds[3 * TOT + o];
                emit(v, o % (P * SW), s);
            }
        }
        __syncthreads();
    }
}

}  // namespace mar
