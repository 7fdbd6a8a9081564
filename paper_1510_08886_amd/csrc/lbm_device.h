// Device-side helpers shared by the 2D channel, 3D duct and batched kernels:
// storage encodings, stochastic rounding, compile-time pair loops, the Hermite
// equilibrium for initial states and FP64 block sums.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>

#include "lbm_internal.h"
#include "lbm_sets.h"

namespace lbm {

// ---------------------------------------------------------------------------
// storage traits: T is the stored type, R the arithmetic type.
//   F64    : fbar in double
//   F32    : d = fbar - w rho0 in float
//   F32RAW : fbar in float
//   F16DEV : kF16Scale d / (w rho0) in half, stochastic rounding in time steps
// ---------------------------------------------------------------------------
// The scale keeps small deviations (a flow started from rest, Ma ~ 1e-3) in
// half's normal range, where stochastic rounding is exact and unbiased; below
// it the conversion rounds to nearest, which biases a uniform field. It bounds
// |d / (w rho0)| by 65504 / 1024 = 64. The tables' wr0 / inv_wr0 carry it.
constexpr double kF16Scale = 1024.0;
template <Storage S>
struct St;
template <>
struct St<Storage::F64> {
    using T = double;
    using R = double;
};
template <>
struct St<Storage::F32> {
    using T = float;
    using R = float;
};
template <>
struct St<Storage::F32RAW> {
    using T = float;
    using R = float;
};
template <>
struct St<Storage::F16DEV> {
    using T = _Float16;
    using R = float;
};
template <>
struct St<Storage::F32SR> {
    using T = float;
    using R = double;
};

// PCG-family integer hash (Jarzynski & Olano, "Hash Functions for GPU
// Rendering", JCGT 2020): one 32-bit output per 32-bit input.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

// Stochastic rounding of a float to half on the magnitude, by the hardware
// conversion of gfx950: the top 13 bits of rnd are added below the half
// mantissa and truncated with it (checked on MI355X on inputs of known
// truncated fraction: the same result as adding rnd >> 19 to the float's bit
// pattern and truncating 13 bits), one instruction instead of three.
__device__ __forceinline__ _Float16 sr_half(float x, uint32_t rnd) {
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const half2_t v = __builtin_amdgcn_cvt_sr_f16_f32(half2_t{}, x, rnd, false);
    return v[0];
}

// Stochastic rounding of a double to float on the magnitude: the 29 mantissa
// bits below float precision get 29 random bits added and are then cleared,
// so the magnitude rounds up with a probability equal to the dropped fraction
// (unbiased), and the cleared double converts to float exactly (normal range).
__device__ __forceinline__ float sr_float(double x, uint32_t rnd) {
    uint64_t b = (uint64_t)__double_as_longlong(x);
    b += (uint64_t)(rnd >> 3);
    b &= ~((uint64_t(1) << 29) - 1);
    return (float)__longlong_as_double((long long)b);
}

template <Storage S>
__device__ __forceinline__ typename St<S>::R decode_dev(typename St<S>::T v,
                                                         typename St<S>::R wr0) {
    using R = typename St<S>::R;
    if constexpr (S == Storage::F16DEV)
        return wr0 * (R)v;
    else if constexpr (S == Storage::F32 || S == Storage::F32SR)
        return (R)v;
    else
        return (R)v - wr0;
}

// SRND selects stochastic rounding for the half and the FP32SR storages (time
// steps); init and import round to nearest so that an exported state
// re-imports bit-exactly.
template <Storage S, bool SRND>
__device__ __forceinline__ typename St<S>::T encode_dev(typename St<S>::R d,
                                                         typename St<S>::R wr0,
                                                         typename St<S>::R inv_wr0,
                                                         uint32_t rnd) {
    using T = typename St<S>::T;
    if constexpr (S == Storage::F16DEV && SRND)
        return sr_half(d * inv_wr0, rnd);
    else if constexpr (S == Storage::F16DEV)
        return (T)(d * inv_wr0);
    else if constexpr (S == Storage::F32SR && SRND)
        return sr_float(d, rnd);
    else if constexpr (S == Storage::F32 || S == Storage::F32SR)
        return (T)d;
    else
        return (T)(d + wr0);
}

// exact FP64 value of a stored population
template <Storage S>
__device__ __forceinline__ double stored_value(typename St<S>::T v, double wrd) {
    if constexpr (S == Storage::F16DEV)
        return wrd * (1.0 + (double)(float)v * (1.0 / kF16Scale));
    else if constexpr (S == Storage::F32 || S == Storage::F32SR)
        return wrd + (double)v;
    else
        return (double)v;
}

// the part of a stored population's FP64 value that varies: the whole value
// for fbar storages, the deviation for deviation storages (whose constant
// w rho0 parts are summed on the host)
template <Storage S>
__device__ __forceinline__ double stored_part(typename St<S>::T v, typename St<S>::R wr0) {
    if constexpr (S == Storage::F16DEV)
        return (double)wr0 * (double)(float)v;
    else
        return (double)v;
}

// Population store of a time step. STREAM selects the non-temporal
// (streaming) hint: the value is not read again in this launch. Measured on
// MI355X: it speeds up the 128x256x256 D3V39 duct (2.6 GB of populations) by
// 4% (FP32) and 8% (FP16), and slows the 2048x512 D2V37 channel (310 MB, close
// to the 256 MB last-level cache that can serve the next step's reads) by 5%.
template <bool STREAM, typename T>
__device__ __forceinline__ void store_pop(T *p, T v) {
    if constexpr (STREAM)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// per-node random word for stochastic rounding (n = solve-local node index)
__device__ __forceinline__ uint32_t node_key(uint32_t n, uint32_t step) {
    return pcg_hash(n ^ pcg_hash(step));
}

// Population storage layout ("AoSoA-64"): nodes are grouped in blocks of 64
// consecutive node indices; a block holds all V populations of its nodes, each
// population as one contiguous 64-entry run. Element (alpha, n) lives at
// (n / 64) * 64 V + 64 alpha + n % 64. A wavefront of 64 consecutive nodes thus
// reads and writes whole 256-byte (FP32) runs, and the populations of one
// block share DRAM pages, which streams far better than one plane per velocity.
template <int V>
__device__ __forceinline__ uint32_t aos_base(uint32_t n) {
    return (n >> 6) * (uint32_t)(64 * V) + (n & 63u);
}

// (x mod n) for x in [-h, n + h)
__device__ __forceinline__ int wrap_col(int x, int n, int h) {
    if (n >= h) {
        x = x < 0 ? x + n : x;
        return x >= n ? x - n : x;
    }
    return ((x % n) + n) % n;
}

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------
template <class F, int... P>
__device__ __forceinline__ void for_pairs_impl(F &&f, std::integer_sequence<int, P...>) {
    (f(std::integral_constant<int, P>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void for_pairs(F &&f) {
    for_pairs_impl(f, std::make_integer_sequence<int, N>{});
}

// acc + E * a for a small compile-time integer E
template <int E, typename R>
__device__ __forceinline__ R addk(R acc, R a) {
    if constexpr (E == 0)
        return acc;
    else if constexpr (E == 1)
        return acc + a;
    else if constexpr (E == -1)
        return acc - a;
    else
        return fma(R(E), a, acc);
}
// E * a
template <int E, typename R>
__device__ __forceinline__ R mulk(R a) {
    if constexpr (E == 1)
        return a;
    else if constexpr (E == -1)
        return -a;
    else
        return R(E) * a;
}
// A x + B y for compile-time integers (0 when both vanish)
template <int A, int B, typename R>
__device__ __forceinline__ R lin2(R x, R y) {
    if constexpr (A == 0 && B == 0)
        return R(0);
    else if constexpr (A == 0)
        return mulk<B>(y);
    else
        return addk<B>(mulk<A>(x), y);
}
template <int A, int B, int C, typename R>
__device__ __forceinline__ R lin3(R x, R y, R z) {
    if constexpr (A == 0)
        return lin2<B, C>(y, z);
    else
        return addk<C>(addk<B>(mulk<A>(x), y), z);
}

// Encode all velocities of one node. Stochastic rounding (time steps of the
// half and FP32SR storages) takes one PCG hash of (node, step) and gives slot
// alpha the top bits (13 for half, 29 for FP32SR) of key + alpha * 0x9E3779B9, a Weyl sequence with the golden-ratio
// increment: each offset is uniform, and the offsets of one node are evenly
// spread rather than independent, which keeps a node's rounding errors from
// adding up. Two operations per slot instead of a hash per slot.
template <class SET, Storage S, bool SRND>
__device__ __forceinline__ void encode_all(const typename St<S>::R (&d)[SET::V],
                                           const PairTable<typename St<S>::R> &t, uint32_t n,
                                           uint32_t step, typename St<S>::T (&v)[SET::V]) {
    constexpr int NR = SET::NR;
    uint32_t key = 0;
    if constexpr (stochastic_storage(S) && SRND) key = node_key(n, step);
    auto rnd = [&](int slot) -> uint32_t { return key + (uint32_t)slot * 0x9E3779B9u; };
    if constexpr (NR) v[0] = encode_dev<S, SRND>(d[0], t.wr00, t.inv_wr00, rnd(0));
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        v[NR + 2 * p] = encode_dev<S, SRND>(d[NR + 2 * p], t.wr0[p], t.inv_wr0[p], rnd(NR + 2 * p));
        v[NR + 2 * p + 1] =
            encode_dev<S, SRND>(d[NR + 2 * p + 1], t.wr0[p], t.inv_wr0[p], rnd(NR + 2 * p + 1));
    });
}

// f^(0) - w rho0 = w [ (rho - rho0) + rho sum_{1<=n<=5} P_n / n! ] with the scalar
// Hermite recurrence P_{n+1} = (u.xi) P_n - n |u|^2 P_{n-1} (u^n : H^(n)(xi)).
template <class SET, typename R>
__device__ __forceinline__ void equilibrium_dev(const PairTable<R> &t, const StepScalars<R> &s,
                                                double rho_d, R ux, R uy, R uz,
                                                R (&d)[SET::V]) {
    constexpr int NR = SET::NR;
    const R drho = (R)(rho_d - s.rho0d);
    const R rho = (R)rho_d;
    const R u2 = ux * ux + uy * uy + uz * uz;
    const R c = t.c;
    if constexpr (NR) d[0] = t.w0 * (drho + rho * (s.cn[2] * (-u2) + s.cn[4] * R(3) * u2 * u2));
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        const R ue = c * (R(SET::EX[p]) * ux + R(SET::EY[p]) * uy + R(SET::EZ[p]) * uz);
        R Pm = 1, P = ue, even = 0, odd = ue;
        for (int k = 1; k < 5; ++k) {
            const R Pn = ue * P - R(k) * u2 * Pm;
            Pm = P;
            P = Pn;
            if ((k + 1) & 1)
                odd += s.cn[k + 1] * P;
            else
                even += s.cn[k + 1] * P;
        }
        d[NR + 2 * p] = t.w[p] * (drho + rho * (even + odd));
        d[NR + 2 * p + 1] = t.w[p] * (drho + rho * (even - odd));
    });
}

// deviations of one node from canonical FP64 populations in[alpha * nodes + n]
template <class SET, typename R>
__device__ __forceinline__ void import_node(const double *in, const PairTable<R> &t,
                                            uint32_t nodes, uint32_t n, R (&d)[SET::V]) {
    constexpr int NR = SET::NR;
    if constexpr (NR) d[0] = (R)(in[n] - t.wrd0);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        d[NR + 2 * p] = (R)(in[(uint32_t)(NR + 2 * p) * nodes + n] - t.wrd[p]);
        d[NR + 2 * p + 1] = (R)(in[(uint32_t)(NR + 2 * p + 1) * nodes + n] - t.wrd[p]);
    });
}

// FP64 sums of (a, b) over a block into partial[2 * blockIdx.x + {0,1}]
__device__ __forceinline__ void block_sum2(double a, double b, double *partial) {
    __shared__ double sa[16], sb[16];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sa[wv] = a;
        sb[wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            ta += sa[w];
            tb += sb[w];
        }
        partial[2 * blockIdx.x] = ta;
        partial[2 * blockIdx.x + 1] = tb;
    }
}

// ---------------------------------------------------------------------------
// raw buffer accesses: a scalar descriptor (base, size in bytes), a per-lane
// 32-bit byte offset and a uniform (scalar) byte offset. Used by the aligned
// step kernels, whose row offsets are uniform, so that an access costs no
// vector address arithmetic. Word 3 of the descriptor selects the 32-bit data
// format of the gfx9 family; accesses beyond `bytes` read 0 and drop stores.
// ---------------------------------------------------------------------------
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}

// STREAM: non-temporal hint (cache policy bit 1)
template <bool STREAM, typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, T v, uint32_t voff,
                                          uint32_t soff) {
    constexpr int aux = STREAM ? 2 : 0;
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, aux);
    else if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff,
                                              aux);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff,
                                              aux);
}

// ---------------------------------------------------------------------------
// node-local accesses of the in-place population array (PopLayout), shared by
// the 2D and 3D kernels
// ---------------------------------------------------------------------------
// Element position split into a per-lane part l, a uniform part u and a slot
// offset o (a compile-time constant once inlined): the flat index is
// l + u + o. Aligned step kernels keep row offsets in u (scalar registers) and
// the column part in l.
struct Ix {
    uint32_t l, u, o;
};
__device__ __forceinline__ Ix slot_of(Ix x, int a) { return {x.l, x.u, x.o + 64u * (uint32_t)a}; }

// flat pointer access
template <typename T>
struct GlobalPop {
    T *A;
    __device__ __forceinline__ T ld(Ix x) const { return A[(x.u + x.l) + x.o]; }
    template <bool STREAM>
    __device__ __forceinline__ void st(Ix x, T v) const {
        store_pop<STREAM>(A + (x.u + x.l) + x.o, v);
    }
    // a position as one flat index (in l)
    static __device__ __forceinline__ Ix flat(Ix x) { return {(x.u + x.l) + x.o, 0u, 0u}; }
};

// raw buffer access (arrays below 2 GiB): the uniform part becomes the scalar
// offset operand
template <typename T>
struct BufferPop {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ BufferPop(const void *p, uint32_t bytes) : r(make_rsrc(p, bytes)) {}
    __device__ __forceinline__ T ld(Ix x) const {
        return buf_load<T>(r, x.l * (uint32_t)sizeof(T), (x.u + x.o) * (uint32_t)sizeof(T));
    }
    template <bool STREAM>
    __device__ __forceinline__ void st(Ix x, T v) const {
        buf_store<STREAM>(r, v, x.l * (uint32_t)sizeof(T), (x.u + x.o) * (uint32_t)sizeof(T));
    }
    // the slot offset folded into the uniform part
    static __device__ __forceinline__ Ix flat(Ix x) { return {x.l, x.u + x.o, 0u}; }
};

// kStreamed -> pre-collision values: slot alpha of the node itself
template <class SET, class P, typename T>
__device__ __forceinline__ void read_local(const P &pop, Ix own, T (&raw)[SET::V]) {
#pragma unroll
    for (int a = 0; a < SET::V; ++a) raw[a] = pop.ld(slot_of(own, a));
}

// post-collision values -> the node's own slots: kLocal (SWAP, velocity alpha
// in the slot of -alpha) or kDirect (slot alpha)
template <class SET, bool SWAP, bool STREAM, class P, typename T>
__device__ __forceinline__ void write_own(const P &pop, Ix own, const T (&v)[SET::V]) {
    constexpr int NR = SET::NR;
    if constexpr (NR) pop.template st<STREAM>(own, v[0]);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        pop.template st<STREAM>(slot_of(own, SWAP ? NR + 2 * p + 1 : NR + 2 * p), v[NR + 2 * p]);
        pop.template st<STREAM>(slot_of(own, SWAP ? NR + 2 * p : NR + 2 * p + 1), v[NR + 2 * p + 1]);
    });
}

template <class SET, bool SWAP, bool STREAM, typename T>
__device__ __forceinline__ void write_own(T *A, uint32_t own, const T (&v)[SET::V]) {
    write_own<SET, SWAP, STREAM>(GlobalPop<T>{A}, Ix{own, 0u, 0u}, v);
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
static inline int hip_ok(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return LBM_OK;
}

static inline unsigned blocks_for(int64_t nodes) { return (unsigned)((nodes + 255) / 256); }

struct Entry {
    int id;
    Storage s;
    const Launch *l;
};

}  // namespace lbm
