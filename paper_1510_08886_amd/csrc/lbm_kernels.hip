// HIP kernels for gfx950: fused pull-stream + diffuse Maxwell wall + BGK
// collision of the modified populations (Eq. nm.8) on 2D channels, plus
// observation, initialisation and population import/export.
//
// Layout in HBM: blocks of 64 consecutive nodes (node n = y * nx + x) with all
// populations of a block together, one contiguous 64-entry run per velocity
// slot (aos_base). A wavefront covers one block; a neighbour access of
// velocity alpha is one run shifted by the velocity, spanning at most two
// blocks of the neighbouring row. One array per solve, updated in place
// (PopLayout).
//
// Kernels are specialised per velocity set (lbm_sets.h): integer velocity
// components are compile-time constants, so moments are integer-weighted sums,
// zero components cost nothing, and source offsets come from per-node tables
// of row and column offsets. Velocities come in pairs (e, -e); the even and odd
// parts of the equilibrium and force are formed once per pair.
//
// Arithmetic: the collision works on deviations d = fbar - w rho0 so that the
// moments of a nearly uniform state do not cancel in FP32.
//
// Wall (Eqs. nm.14, nm.15, transformed to fbar): an unknown population at node
// x is rho_eff(e) w (1 - dt/2 g.xi), with rho_eff(e) = A(e) / D(e); A(e) is the
// FP64 sum of the post-collision populations that crossed the wall at element e
// in this streaming step. A step writes, per wall row r < HN and column, the
// FP64 partial of the populations it has just stored that leave through the
// wall next step; the next step sums the partials of its column. The element
// is the column of the fluid node next to the crossing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "lbm_node2d.h"

namespace lbm {

// ---------------------------------------------------------------------------
// One population array per solve (the AA pattern; two layouts, see
// PopLayout). A step reads and writes the same set of locations per node, so
// nodes never race, and the update runs in place: half the memory of a
// ping-pong pair, and for arrays that fit the 256 MB last-level cache the next
// step is largely served from it.
//
// Neighbour addressing of node (i, j): position of slot 0 of node
// (j - dy, i - dx), |dy| <= HN, |dx| <= H, rows clamped into the channel (so
// every address is valid), columns periodic. ALIGNED (nx % 64 == 0): a row is
// a whole number of 64-node blocks, so the index is a row part (uniform when
// the row is) plus a column part.
// ---------------------------------------------------------------------------
template <class SET, bool ALIGNED>
struct Nbr2 {
    static constexpr int H = SET::H, HN = SET::HN, V = SET::V;
    int rows[2 * HN + 1];
    uint32_t col[2 * H + 1];
    uint32_t rowstride;
    int nx;
    template <class SC>
    __device__ __forceinline__ Nbr2(const SC &s, int i, int j) : nx(s.nx) {
        rowstride = (uint32_t)s.nx * V;
#pragma unroll
        for (int k = -HN; k <= HN; ++k) rows[k + HN] = min(max(j - k, 0), s.ny - 1);
#pragma unroll
        for (int k = -H; k <= H; ++k) {
            const uint32_t x = (uint32_t)wrap_col(i - k, s.nx, H);
            col[k + H] = ALIGNED ? (x >> 6) * (uint32_t)(64 * V) + (x & 63u) : x;
        }
    }
    __device__ __forceinline__ Ix at(int dy, int dx) const {
        if constexpr (ALIGNED)
            return {col[dx + H], (uint32_t)rows[dy + HN] * rowstride, 0u};
        else
            return {aos_base<V>((uint32_t)rows[dy + HN] * (uint32_t)nx + col[dx + H]), 0u, 0u};
    }
};

// Pull of the pre-collision values from the neighbours: population +e_p of x
// comes from x - e_p, in slot -e_p (SWAP, kLocal) or slot +e_p (kDirect).
// Rows are clamped: a wall slot reads a valid, unused value that complete2d
// replaces.
template <class SET, bool SWAP, class NB, class P, typename T>
__device__ __forceinline__ void read_pull(const P &pop, const NB &nb, Ix own, T (&raw)[SET::V]) {
    constexpr int NR = SET::NR;
    if constexpr (NR) raw[0] = pop.ld(own);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int ex = SET::EX[p], ey = SET::EY[p];
        raw[NR + 2 * p] = pop.ld(slot_of(nb.at(ey, ex), SWAP ? NR + 2 * p + 1 : NR + 2 * p));
        raw[NR + 2 * p + 1] = pop.ld(slot_of(nb.at(-ey, -ex), SWAP ? NR + 2 * p : NR + 2 * p + 1));
    });
}

// Home of post-collision population +e_p (PLUS) or -e_p of node x in the
// kStreamed layout: slot +-e_p of the destination x +- e_p, or, when that lies
// outside the channel, the node's own slot of the opposite velocity.
// INTERIOR: the node is at least HN rows from both walls (every destination
// inside).
template <class SET, int p, bool PLUS, bool INTERIOR, class P, class NB>
__device__ __forceinline__ Ix home2d(const NB &nb, Ix own, int j, int ny) {
    constexpr int NR = SET::NR, ex = SET::EX[p], ey = SET::EY[p];
    constexpr int sy = PLUS ? ey : -ey, sx = PLUS ? ex : -ex;
    constexpr int slot = PLUS ? NR + 2 * p : NR + 2 * p + 1, opp = PLUS ? NR + 2 * p + 1 : NR + 2 * p;
    if constexpr (sy == 0 || INTERIOR) {
        return slot_of(nb.at(-sy, -sx), slot);
    } else {
        const bool inside = (unsigned)(j + sy) < (unsigned)ny;
        const Ix there = slot_of(nb.at(-sy, -sx), slot), here = slot_of(own, opp);
        return inside ? P::flat(there) : P::flat(here);
    }
}

// post-collision values -> kStreamed layout
template <class SET, bool STREAM, bool INTERIOR, class NB, class P, typename T>
__device__ __forceinline__ void write_gs(const P &pop, const NB &nb, Ix own, int j, int ny,
                                         const T (&v)[SET::V]) {
    constexpr int NR = SET::NR;
    if constexpr (NR) pop.template st<STREAM>(own, v[0]);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        pop.template st<STREAM>(home2d<SET, p, true, INTERIOR, P>(nb, own, j, ny), v[NR + 2 * p]);
        pop.template st<STREAM>(home2d<SET, p, false, INTERIOR, P>(nb, own, j, ny), v[NR + 2 * p + 1]);
    });
}

// Step kinds: the ping-pong pull (kDirect in pop, kDirect out to pop_out), and
// the two in-place kinds (kLocal -> gather/scatter -> kStreamed; kStreamed ->
// node-local -> kLocal).
enum StepKind : int { kPingPong = 0, kGatherScatter = 1, kNodeLocal = 2 };

template <class SET, Storage S, bool ALIGNED, bool STREAM, int KIND, bool N5>
__device__ __forceinline__ void step_node2d(const StepBuffers &b,
                                            const PairTable<typename St<S>::R> &t,
                                            const StepScalars<typename St<S>::R> &s,
                                            uint32_t step, int i, int j, uint32_t n);

// One thread per node, blocks of up to 256 threads: one block per (x tile,
// row) when rows are whole 64-node blocks, else per 256 consecutive nodes.
// Each thread issues all its loads before it decodes any, so a wavefront has
// its whole gather in flight at once; wall slots are patched after the loads.
// The host runs arrays of up to 512 MiB in place (on MI355X ~7% faster than
// ping-pong for the 155 MB D2V37 channel: the array stays largely in the
// 256 MB last-level cache) and larger ones ping-pong (10-14% faster at
// 1.2-1.3 GB). Also measured and rejected: a persistent grid with a two-stage
// register load pipeline (occupancy 2), a persistent grid streaming the next
// tile's gather into LDS with global_load_lds (LDS-limited to 8 waves per CU),
// 64-, 128- and 512-node tiles, register caps for 6 to 8 waves per SIMD.
template <class SET, Storage S, bool ALIGNED, bool STREAM, int KIND, bool N5>
__global__ __launch_bounds__(256)
void k_step2d(StepBuffers b, PairTable<typename St<S>::R> t, StepScalars<typename St<S>::R> s,
              uint32_t step) {
    // ALIGNED: a 2D grid of (x tile, row) blocks, so the row, and every row
    // offset, is uniform (scalar registers); otherwise 256 consecutive nodes
    int i, j;
    uint32_t n;
    if constexpr (ALIGNED) {
        // Workgroups go to the 8 XCDs round-robin by linear id. XCD x takes
        // the k-th of its workgroups from a contiguous band of tiles in row
        // order (x * (total / 8) + min(x, total % 8) + k), so the cache lines
        // two adjacent tiles of a row share (shifted runs) stay in one L2.
        // The upper four bands run backwards, so that the slower wall rows at
        // the top of the channel come first, as those at the bottom do, and
        // not at the end of the launch (measured 2% faster).
        // The node-local kind, which always follows a gather/scatter step,
        // walks every band the other way, so it starts on the tiles the
        // previous step touched last, which are still in that XCD's L2 (a
        // 16 MB copy between steps removes the gain); the two wall bands
        // first take their HN wall rows, then the rest of the band in that
        // opposite direction. Measured on MI355X: D2V37 44.4 -> 43.0 us and
        // D2V32 40.7 -> 39.9 us per step; reversing the wall bands too, wall
        // rows last, gave 43.9 and 41.2 us.
        const uint32_t tiles = gridDim.x, total = tiles * gridDim.y;
        const uint32_t id = blockIdx.y * tiles + blockIdx.x, xcd = id & 7u;
        const uint32_t cnt = (total >> 3) + (xcd < (total & 7u) ? 1u : 0u);
        const uint32_t q = id >> 3;
        uint32_t k = xcd >= 4u ? cnt - 1u - q : q;
        if constexpr (KIND == kNodeLocal) {
            const uint32_t w = (xcd == 0u || xcd == 7u) ? min(cnt, (uint32_t)SET::HN * tiles) : 0u;
            if (q >= w) k = xcd >= 4u ? q - w : cnt - 1u - (q - w);
        }
        const uint32_t lin = xcd * (total >> 3) + min(xcd, total & 7u) + k;
        j = (int)(lin / tiles);
        i = (int)((lin - (uint32_t)j * tiles) * blockDim.x + threadIdx.x);
        n = (uint32_t)j * (uint32_t)s.nx + (uint32_t)i;
    } else {
        n = blockIdx.x * 256u + threadIdx.x;
        if (n >= (uint32_t)s.nodes) return;
        j = (int)(n / (uint32_t)s.nx);
        i = (int)(n - (uint32_t)j * s.nx);
    }
    step_node2d<SET, S, ALIGNED, STREAM, KIND, N5>(b, t, s, step, i, j, n);
}

// One step of node n = (j, i): pull (or read own slots), wall fill, moments,
// relaxation, store, wall partials.
template <class SET, Storage S, bool ALIGNED, bool STREAM, int KIND, bool N5>
__device__ __forceinline__ void step_node2d(const StepBuffers &b,
                                            const PairTable<typename St<S>::R> &t,
                                            const StepScalars<typename St<S>::R> &s,
                                            uint32_t step, int i, int j, uint32_t n) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    // BUF (aligned rows; 16-bit storage, or stencils reaching 7 or more
    // columns): raw buffer accesses with the row and slot offsets in the
    // scalar operand (arrays below 2 GiB), which removes the vector address
    // arithmetic. Measured on MI355X: 4% faster for the FP16 duct step, whose
    // arithmetic outweighs its halved traffic, and 3% for the FP32 D2V32
    // channel (25 column offsets); 0.4-2% slower for the FP32 D2V37 step (the
    // compiler then batches the stores after the collision instead of
    // interleaving them), which keeps flat addresses.
    constexpr bool BUF = ALIGNED && (sizeof(T) == 2 || SET::H >= kBufferMinHalo);
    T *A = (T *)b.pop;
    auto pop_at = [&](void *base) {
        if constexpr (BUF)
            return BufferPop<T>(base, (uint32_t)s.nodes * (uint32_t)(SET::V * sizeof(T)));
        else
            return GlobalPop<T>{(T *)base};
    };
    const auto pop = pop_at(A);
    const Ix own = BUF ? Ix{((uint32_t)i >> 6) * (uint32_t)(64 * SET::V) + ((uint32_t)i & 63u),
                                (uint32_t)j * (uint32_t)s.nx * SET::V, 0u}
                       : Ix{aos_base<SET::V>(n), 0u, 0u};
    T raw[SET::V];
    // KIND == kNodeLocal reads only the node's own slots
    const Nbr2<SET, ALIGNED> nb(s, i, j);
    // Wide stencils issue their reads at raised wavefront priority, so that
    // waves still issuing loads go ahead of waves in their collision: measured
    // on MI355X, D2V32 41.2 -> 40.7 us per step. For D2V37 the node-local kind
    // gained 1% with it until its tiles ran in the alternating band order,
    // and nothing since; its gather/scatter kind lost 4%.
    constexpr bool PRIO = SET::H >= kBufferMinHalo;
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
    if constexpr (KIND == kNodeLocal)
        read_local<SET>(pop, own, raw);
    else
        read_pull<SET, KIND == kGatherScatter>(pop, nb, own, raw);
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    R d[SET::V];
    // specular walls (accommodation < 1) are stepped ping-pong only
    if constexpr (KIND == kPingPong)
        complete2d<SET, S>(raw, b.a_cur, t, s, i, j, d, ArrayMirror<SET, T>{(const T *)b.pop, i, s.nx});
    else
        complete2d<SET, S>(raw, b.a_cur, t, s, i, j, d);
    relax2d<SET, R, N5>(d, t, s, t.c);
    T v[SET::V];
    encode_all<SET, S, true>(d, t, n, step, v);
    if constexpr (KIND == kGatherScatter && BUF) {
        // Each write position equals another velocity's read position: 2H + 1
        // column offsets stay live (rows are scalar). Rows at least HN from
        // both walls (a uniform test) store without the wall selects.
        if (j >= SET::HN && j < s.ny - SET::HN)
            write_gs<SET, STREAM, true>(pop, nb, own, j, s.ny, v);
        else
            write_gs<SET, STREAM, false>(pop, nb, own, j, s.ny, v);
    } else if constexpr (KIND == kGatherScatter) {
        // Flat addresses: an opaque copy of (i, j) makes the compiler recompute
        // the write addresses here instead of keeping ~V 64-bit addresses
        // live through the collision.
        int iw = i, jw = j;
        asm volatile("" : "+v"(iw), "+v"(jw));
        const Nbr2<SET, ALIGNED> nbw(s, iw, jw);
        write_gs<SET, STREAM, false>(pop, nbw, own, jw, s.ny, v);
    } else if constexpr (KIND == kNodeLocal) {
        write_own<SET, true, STREAM>(pop, own, v);
    } else {
        write_own<SET, false, STREAM>(pop_at(b.pop_out), own, v);
    }
    wall_partials2d<SET, S>(v, t, s, i, j, b.a_next);
}

// Many in-place steps of a small problem (at most kResidentMaxNodes nodes) in
// one workgroup: each step runs the per-node code of k_step2d over all nodes
// (threads loop over nodes), the two in-place kinds alternate, and a workgroup
// barrier, which orders the global stores and loads of the workgroup's waves
// on their common CU, separates consecutive steps. One launch thus replaces
// nsteps dependent launches and their device-side latency; the arithmetic and
// the results are those of one launch per step.
template <class SET, Storage S, bool N5>
__global__ __launch_bounds__(256) void k_run2d(StepBuffers b, PairTable<typename St<S>::R> t,
                                               StepScalars<typename St<S>::R> s, uint32_t step0,
                                               int nsteps) {
    const double *a_cur = b.a_cur;
    double *a_next = b.a_next;
    int layout = b.layout;
    for (int k = 0; k < nsteps; ++k) {
        StepBuffers bk = b;
        bk.layout = layout;
        bk.a_cur = a_cur;
        bk.a_next = a_next;
        for (uint32_t n = threadIdx.x; n < (uint32_t)s.nodes; n += blockDim.x) {
            const int j = (int)(n / (uint32_t)s.nx);
            const int i = (int)(n - (uint32_t)j * s.nx);
            if (layout == kLocal)
                step_node2d<SET, S, false, false, kGatherScatter, N5>(bk, t, s, step0 + k, i, j, n);
            else
                step_node2d<SET, S, false, false, kNodeLocal, N5>(bk, t, s, step0 + k, i, j, n);
        }
        __syncthreads();
        double *const written = a_next;
        a_next = const_cast<double *>(a_cur);
        a_cur = written;
        layout = layout == kLocal ? kStreamed : kLocal;
    }
}

// ---------------------------------------------------------------------------
// Two ping-pong steps per launch (temporal blocking). A workgroup owns a tile
// of BX columns of a band of rows and sweeps it upwards in chunks of RR rows.
// Step t is computed for the tile widened by the stencil reach (H columns and
// HN rows on each side, the extra nodes computed by both neighbours), from
// the source copy in HBM, and kept in a ring of RR + 2 HN rows in LDS; step
// t + 1 of each chunk then pulls from the ring and goes to the destination
// copy. Per two lattice updates a node is thus read once and written once in
// HBM. Workgroups never exchange data, so nothing waits on another workgroup;
// inside one, barriers order the ring's writes and reads. The per-node
// arithmetic, the stochastic-rounding keys and the FP64 wall partials are
// those of two kPingPong launches, so the results are bit for bit the same.
//
// The wall partials that step t writes for step t + 1 (only the tile's own
// columns are ever needed) stay in LDS: a band touching a wall computes all of
// that wall's rows in step t (its widened rows reach them), so every wall row
// of step t + 1 finds its column's partials.
// ---------------------------------------------------------------------------
// Two schedules, both one workgroup per CU (the ring takes most of the LDS):
//   kPairAlternate: all waves compute step t of a chunk of RR rows, a barrier,
//     then all compute step t + 1 of the chunk (ring of RR + 2 HN rows);
//   kPairSplit: producer waves compute step t of chunk k + 1 while consumer
//     waves compute step t + 1 of chunk k (ring of 2 RR + 2 HN rows), so the
//     HBM reads of one overlap the arithmetic of the other. The two groups
//     hand over chunks through two LDS counters (release / acquire at
//     workgroup scope); a workgroup's waves are resident together, so every
//     wait ends. Each wait is also bounded: one that gives up raises a flag in
//     device memory (read by the host at the next observation) and its wave
//     leaves, and so, in turn, does the other group's.
//   kPairTwin: as kPairSplit, with two producer groups that take the even and
//     the odd chunks. A producer gathers and collides its chunk before it
//     waits for the ring rows to be free, and only its ring writes wait, so
//     the gather of one group is in flight while the other computes: with a
//     single group each chunk's HBM latency lies on the critical path. Chunks
//     of fewer rows keep the waves at three per SIMD, the register budget of
//     the single-group form.
enum PairKind : int { kPairAlternate = 1, kPairSplit = 2, kPairTwin = 3 };

template <class SET, typename T, int KIND>
struct PairTile {
    static constexpr int H = SET::H, HN = SET::HN, V = SET::V;
    static constexpr size_t kLds = 156 * 1024;     // of the 160 KB of a gfx950 CU
    // ring rows for chunks of rr rows
    static constexpr int ring_rows(int rr) { return (KIND == kPairAlternate ? 1 : 2) * rr + 2 * HN; }
    static constexpr size_t bytes(int bx, int rr) {
        return (size_t)ring_rows(rr) * (bx + 2 * H) * V * sizeof(T) + (size_t)2 * HN * bx * 8;
    }
    static constexpr int up64(int x) { return (x + 63) / 64 * 64; }
    // threads: one step-t node of a chunk each (per producer group) and, for
    // the split kinds, one step-(t+1) node of a chunk each, in waves of their
    // own
    static constexpr int threads(int bx, int rr) {
        return up64(rr * (bx + 2 * H)) * (KIND == kPairTwin ? 2 : 1) +
               (KIND == kPairAlternate ? 0 : up64(rr * bx));
    }
    // kPairTwin: at most three waves per SIMD (12 per CU), so that each wave
    // keeps 168 VGPRs
    static constexpr int kMaxThreads = KIND == kPairTwin ? 768 : 1024;
    static constexpr bool fits(int bx, int rr) {
        return bytes(bx, rr) <= kLds && threads(bx, rr) <= kMaxThreads;
    }
    static constexpr int pick_bx() {
        return fits(64, KIND == kPairAlternate ? 8 : KIND == kPairSplit ? 4 : 3) ? 64 : 32;
    }
    static constexpr int pick_rr(int bx) {
        return fits(bx, 16) ? 16 : fits(bx, 8) ? 8 : fits(bx, 6) ? 6 : fits(bx, 4) ? 4
               : (KIND == kPairTwin && fits(bx, 3)) ? 3 : 2;
    }
    static constexpr int BX = pick_bx();
    static constexpr int RR = pick_rr(BX);
    static constexpr int EW = BX + 2 * H;          // ring row pitch (columns)
    static constexpr int RING = ring_rows(RR);
    static constexpr bool ok = fits(BX, RR) && H <= 4;
    static constexpr int PT = up64(RR * EW);       // threads of one producer group
    static constexpr int NPG = KIND == kPairTwin ? 2 : 1;
    static constexpr int CT = KIND == kPairAlternate ? 0 : up64(RR * BX);
    static constexpr int NT = NPG * PT + CT;
};

// bound of one wait on the other group (~0.5 s): only a broken schedule reaches it
constexpr uint32_t kPairSpinLimit = 1u << 23;

__device__ __forceinline__ bool pair_wait(const int *cnt, int target, int *err) {
    for (uint32_t k = 0;; ++k) {
        if (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= target)
            return true;
        if (k >= kPairSpinLimit) {
            if (err) *err = 1;
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <class SET, Storage S, bool ALIGNED, bool STREAM, bool N5, int KIND>
__global__ __launch_bounds__((PairTile<SET, typename St<S>::T, KIND>::NT))
void k_pair2d(StepBuffers b, PairTable<typename St<S>::R> t, StepScalars<typename St<S>::R> s,
              uint32_t step, int band_rows) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    using TL = PairTile<SET, T, KIND>;
    constexpr int H = SET::H, HN = SET::HN, V = SET::V, NR = SET::NR;
    constexpr int BX = TL::BX, RR = TL::RR, EW = TL::EW, RING = TL::RING;
    __shared__ T ring[RING * V * EW];      // [row mod RING][alpha][column]
    __shared__ double ap[2 * HN * BX];     // step-t partials of the tile's columns [face][row][col]
    // split kinds: waves done per group, summed over the group's chunks
    // (kPairTwin: produced[g] for the producer group of the chunks k = g mod 2)
    __shared__ int produced[2], consumed;

    // tile of this workgroup: XCD x (workgroups go to the 8 XCDs round-robin)
    // takes a contiguous run of tiles in (band, strip) order, so the strips
    // that share halo columns share an L2
    const int nx = s.nx, ny = s.ny;
    const uint32_t total = gridDim.x, id = blockIdx.x, xcd = id & 7u;
    const uint32_t lin = xcd * (total >> 3) + min(xcd, total & 7u) + (id >> 3);
    const int nstrips = (nx + BX - 1) / BX;
    const int strip = (int)(lin % (uint32_t)nstrips), band = (int)(lin / (uint32_t)nstrips);
    const int x0 = strip * BX, ncols = min(BX, nx - x0);
    const int y0 = band * band_rows, y1 = min(y0 + band_rows, ny);
    const int a = max(y0 - HN, 0);         // first step-t row of the band
    const GlobalPop<T> src{(T *)b.pop};
    const GlobalPop<T> dst{(T *)b.pop_out};

    // ring slot of row `row` given the slot sl0 of row r0, |row - r0| < RING
    auto slot_from = [](int sl0, int r0, int row) {
        int x = sl0 + (row - r0);
        x = x < 0 ? x + RING : x;
        return x >= RING ? x - RING : x;
    };
    // step t of rows [lo, hi), columns x0 - H .. x0 + ncols + H - 1, into the
    // ring; threads tid, tid + nth, ... Each node is gathered and collided
    // first; gate() is called before its results go to LDS (kPairTwin: the
    // wait for the ring rows to be free). False when a gate gave up.
    auto first = [&](int lo, int hi, int tid, int nth, auto gate) -> bool {
        const int w = ncols + 2 * H;
        const int n1 = (hi - lo) * w;
        const int sl = (lo - a) % RING;
        for (int e = tid; e < n1; e += nth) {
            const int rl = e / w, c = e - rl * w;
            const int j = lo + rl;
            const int i = wrap_col(x0 - H + c, nx, H);
            const uint32_t n = (uint32_t)j * (uint32_t)nx + (uint32_t)i;
            T raw[V];
            {
                const Nbr2<SET, ALIGNED> nb(s, i, j);
                read_pull<SET, false>(src, nb, Ix{aos_base<V>(n), 0u, 0u}, raw);
            }
            R d[V];
            complete2d<SET, S>(raw, b.a_cur, t, s, i, j, d, ArrayMirror<SET, T>{(const T *)b.pop, i, nx});
            relax2d<SET, R, N5>(d, t, s, t.c);
            T v[V];
            encode_all<SET, S, true>(d, t, n, step, v);
            if (!gate()) return false;
            T *rw = ring + slot_from(sl, lo, j) * (V * EW) + c;
#pragma unroll
            for (int q = 0; q < V; ++q) rw[q * EW] = v[q];
            if (c >= H && c < H + ncols) wall_partials2d_col<SET, S>(v, t, s, j, ap + (c - H), BX);
        }
        return true;
    };
    auto open = [] { return true; };
    // step t + 1 of rows [lo, hi), the tile's own columns, from the ring to HBM
    auto second = [&](int lo, int hi, int tid, int nth) {
        const int n2 = (hi - lo) * BX;
        const int sl = (lo - a) % RING;
        for (int e = tid; e < n2; e += nth) {
            const int rl = e / BX, il = e - rl * BX;
            if (il >= ncols) continue;
            const int j = lo + rl, i = x0 + il;
            const uint32_t n = (uint32_t)j * (uint32_t)nx + (uint32_t)i;
            // ring position of column il + H in the rows j - k, clamped into
            // the channel as the HBM pull clamps them (a wall slot reads a
            // valid value that complete2d_col replaces)
            const T *rb[2 * HN + 1];
#pragma unroll
            for (int k = -HN; k <= HN; ++k) {
                const int jr = min(max(j - k, 0), ny - 1);
                rb[k + HN] = ring + slot_from(sl, lo, jr) * (V * EW) + il + H;
            }
            T raw[V];
            if constexpr (NR) raw[0] = rb[HN][0];
            for_pairs<SET::NP>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                constexpr int ex = SET::EX[p], ey = SET::EY[p];
                raw[NR + 2 * p] = rb[ey + HN][(NR + 2 * p) * EW - ex];
                raw[NR + 2 * p + 1] = rb[HN - ey][(NR + 2 * p + 1) * EW + ex];
            });
            // specular partners from the ring (rows next to a wall are in it)
            auto ring_mirror = [&](int slot, int jm, int ex) -> T {
                return ring[slot_from(sl, lo, jm) * (V * EW) + mirror_slot<SET>(slot) * EW + il + H - ex];
            };
            R d[V];
            complete2d_col<SET, S>(raw, ap + il, BX, t, s, j, d, ring_mirror);
            relax2d<SET, R, N5>(d, t, s, t.c);
            T v[V];
            encode_all<SET, S, true>(d, t, n, step + 1u, v);
            write_own<SET, false, STREAM>(dst, Ix{aos_base<V>(n), 0u, 0u}, v);
            wall_partials2d<SET, S>(v, t, s, i, j, b.a_next);
        }
    };
    // step-t rows chunk k needs: [a, need(k))
    auto need = [&](int k) { return min(y0 + (k + 1) * RR + HN, min(y1 + HN, ny)); };
    const int chunks = (y1 - y0 + RR - 1) / RR;

    if constexpr (KIND == kPairAlternate) {
        for (int k = 0; k < chunks; ++k) {
            first(k == 0 ? a : need(k - 1), need(k), threadIdx.x, blockDim.x, open);
            __syncthreads();
            second(y0 + k * RR, min(y0 + (k + 1) * RR, y1), threadIdx.x, blockDim.x);
            __syncthreads();
        }
    } else {
        static_assert(TL::NT <= TL::kMaxThreads, "producer and consumer waves fit one workgroup");
        constexpr int PW = TL::PT / 64, CW = TL::CT / 64, NPG = TL::NPG;
        if (threadIdx.x == 0) {
            produced[0] = 0;
            produced[1] = 0;
            consumed = 0;
        }
        __syncthreads();
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        // Chunk k is produced by group g = k mod NPG, as that group's
        // (k / NPG)-th chunk. A wave counts a chunk of its group only once
        // every wave of the group has counted the group's previous chunk, so
        // produced[g] >= PW (m + 1) means that all waves of group g have
        // finished the group's m-th chunk (a fast wave cannot stand in for a
        // slow one), and likewise for consumed.
        if (wave < NPG * PW) {
            const int g = wave / PW;
            const int tid = threadIdx.x - g * TL::PT;
            // chunk k overwrites the ring rows of chunk k - 2
            for (int k = g; k < chunks; k += NPG) {
                const int lo = k == 0 ? a : need(k - 1);
                bool ok;
                if constexpr (KIND == kPairTwin) {
                    // gather and collide first; only the ring writes wait
                    ok = first(lo, need(k), tid, TL::PT,
                               [&] { return k < 2 || pair_wait(&consumed, CW * (k - 1), b.err); });
                } else {
                    ok = k < 2 || pair_wait(&consumed, CW * (k - 1), b.err);
                    if (ok) ok = first(lo, need(k), tid, TL::PT, open);
                }
                if (!ok || !pair_wait(&produced[g], PW * (k / NPG), b.err)) return;
                if (lane == 0)
                    __hip_atomic_fetch_add(&produced[g], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        } else {
            for (int k = 0; k < chunks; ++k) {
                if (!pair_wait(&produced[k % NPG], PW * (k / NPG + 1), b.err)) return;
                second(y0 + k * RR, min(y0 + (k + 1) * RR, y1), threadIdx.x - NPG * TL::PT, TL::CT);
                if (!pair_wait(&consumed, CW * k, b.err)) return;
                if (lane == 0)
                    __hip_atomic_fetch_add(&consumed, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// observation: moments of the streamed state, FP64 partial sums per block
// ---------------------------------------------------------------------------
template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_observe2d(const void *pop, int layout, const double *a_cur,
                                                   double *rho_out, double *u_out, double *partial,
                                                   PairTable<typename St<S>::R> t,
                                                   StepScalars<typename St<S>::R> s) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    double ux_d = 0.0, rho_d = 0.0;
    if (n < (uint32_t)s.nodes) {
        const int j = (int)(n / (uint32_t)s.nx);
        const int i = (int)(n - (uint32_t)j * s.nx);
        const GlobalPop<T> A{(T *)pop};
        const Ix own{aos_base<SET::V>(n), 0u, 0u};
        T raw[SET::V];
        if (layout == kStreamed) {
            read_local<SET>(A, own, raw);
        } else {
            const Nbr2<SET, false> nb(s, i, j);
            if (layout == kLocal)
                read_pull<SET, true>(A, nb, own, raw);
            else
                read_pull<SET, false>(A, nb, own, raw);
        }
        R d[SET::V];
        // (specular walls only occur in the ping-pong layout, kDirect)
        complete2d<SET, S>(raw, a_cur, t, s, i, j, d, ArrayMirror<SET, T>{(const T *)pop, i, s.nx});
        const auto m = moments2d<SET, R>(d, s, t.c);
        rho_d = s.rho0d + (double)m.drho;
        ux_d = (double)m.ux;
        if (rho_out) rho_out[n] = rho_d;
        if (u_out) {
            u_out[3 * n] = (double)m.ux;
            u_out[3 * n + 1] = (double)m.uy;
            u_out[3 * n + 2] = 0.0;
        }
    }
    block_sum2(ux_d, rho_d, partial);
}

// ---------------------------------------------------------------------------
// init / import (write the node's own slots: kLocal or kDirect) and export
// ---------------------------------------------------------------------------
template <class SET, Storage S>
__device__ __forceinline__ void store_own2d(typename St<S>::T *A, int layout, double *a_out,
                                            const PairTable<typename St<S>::R> &t,
                                            const StepScalars<typename St<S>::R> &s, int i, int j,
                                            const typename St<S>::R (&d)[SET::V], uint32_t step) {
    using T = typename St<S>::T;
    const uint32_t n = (uint32_t)j * s.nx + i;
    T v[SET::V];
    encode_all<SET, S, false>(d, t, n, step, v);
    if (layout == kLocal)
        write_own<SET, true, false>(A, aos_base<SET::V>(n), v);
    else
        write_own<SET, false, false>(A, aos_base<SET::V>(n), v);
    wall_partials2d<SET, S>(v, t, s, i, j, a_out);
}

template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_init2d(void *dst, int layout, double *a_out,
                                                const double *rho_in, const double *u_in,
                                                PairTable<typename St<S>::R> t,
                                                StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    const int j = (int)(n / (uint32_t)s.nx);
    const int i = (int)(n - (uint32_t)j * s.nx);
    const double rho = rho_in ? rho_in[n] : s.rho0d;
    R ux = 0, uy = 0;
    if (u_in) {
        ux = (R)u_in[3 * n];
        uy = (R)u_in[3 * n + 1];
    }
    R d[SET::V];
    equilibrium_dev<SET, R>(t, s, rho, ux, uy, R(0), d);
    store_own2d<SET, S>((T *)dst, layout, a_out, t, s, i, j, d, step);
}

template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_import2d(void *dst, int layout, double *a_out,
                                                  const double *in, PairTable<typename St<S>::R> t,
                                                  StepScalars<typename St<S>::R> s, uint32_t step) {
    using R = typename St<S>::R;
    using T = typename St<S>::T;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    const int j = (int)(n / (uint32_t)s.nx);
    const int i = (int)(n - (uint32_t)j * s.nx);
    R d[SET::V];
    import_node<SET, R>(in, t, (uint32_t)s.nodes, n, d);
    store_own2d<SET, S>((T *)dst, layout, a_out, t, s, i, j, d, step);
}

// canonical FP64 export [alpha][node] of the post-collision populations
template <class SET, Storage S>
__global__ __launch_bounds__(256) void k_export2d(const void *pop, int layout, double *out,
                                                  PairTable<typename St<S>::R> t,
                                                  StepScalars<typename St<S>::R> s) {
    using T = typename St<S>::T;
    constexpr int NR = SET::NR;
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (uint32_t)s.nodes) return;
    const int j = (int)(n / (uint32_t)s.nx);
    const int i = (int)(n - (uint32_t)j * s.nx);
    const uint32_t nodes = (uint32_t)s.nodes;
    const GlobalPop<T> A{(T *)pop};
    const Ix own{aos_base<SET::V>(n), 0u, 0u};
    const Nbr2<SET, false> nb(s, i, j);
    if constexpr (NR) out[n] = stored_value<S>(A.ld(own), t.wrd0);
    for_pairs<SET::NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        Ix hp, hm;
        if (layout == kLocal) {
            hp = slot_of(own, NR + 2 * p + 1);
            hm = slot_of(own, NR + 2 * p);
        } else if (layout == kDirect) {
            hp = slot_of(own, NR + 2 * p);
            hm = slot_of(own, NR + 2 * p + 1);
        } else {
            hp = home2d<SET, p, true, false, GlobalPop<T>>(nb, own, j, s.ny);
            hm = home2d<SET, p, false, false, GlobalPop<T>>(nb, own, j, s.ny);
        }
        out[(uint32_t)(NR + 2 * p) * nodes + n] = stored_value<S>(A.ld(hp), t.wrd[p]);
        out[(uint32_t)(NR + 2 * p + 1) * nodes + n] = stored_value<S>(A.ld(hm), t.wrd[p]);
    });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Default two-step schedule: two producer groups unless their chunks are
// more than one row shorter than the single group's. Measured on MI355X, 200
// steps per ping-pong copy above the cache (us per step, mode 2 -> mode 3):
// D2V37 FP32 4096 x 2048 (chunks of 4 -> 3 rows) 269 -> 230, D2V37 FP64
// 2048 x 1024 (4 -> 4) 147 -> 136, D2V17 FP32 4096 x 4096 (6 -> 3) 250 -> 268.
template <class SET, typename T>
constexpr bool pair_twin_default() {
    using TW = PairTile<SET, T, kPairTwin>;
    using SP = PairTile<SET, T, kPairSplit>;
    return TW::ok && (!SP::ok || TW::RR + 1 >= SP::RR);
}

template <class SET, Storage S>
struct L2 {
    using R = typename St<S>::R;
    template <int KIND, bool N5>
    static void launch_kind(const StepBuffers &b, const PairTable<R> &t, const StepScalars<R> &s,
                            hipStream_t st, uint32_t stp) {
        const dim3 g(blocks_for(s.nodes)), bl(256);
        // aligned rows: blocks of up to 256 nodes of one row (nx % 64 == 0)
        const unsigned tb = s.nx % 256 == 0 ? 256u : (s.nx % 128 == 0 ? 128u : 64u);
        const dim3 g2((unsigned)s.nx / tb, (unsigned)s.ny), bl2(tb);
        if (s.aligned_rows && s.stream_stores)
            hipLaunchKernelGGL((k_step2d<SET, S, true, true, KIND, N5>), g2, bl2, 0, st, b, t, s, stp);
        else if (s.aligned_rows)
            hipLaunchKernelGGL((k_step2d<SET, S, true, false, KIND, N5>), g2, bl2, 0, st, b, t, s,
                               stp);
        else
            hipLaunchKernelGGL((k_step2d<SET, S, false, false, KIND, N5>), g, bl, 0, st, b, t, s,
                               stp);
    }
    // Hermite order 5 (cn[5] != 0) is compiled for sets of quadrature order 9
    template <int KIND>
    static void launch_step(const StepBuffers &b, const PairTable<R> &t, const StepScalars<R> &s,
                            hipStream_t st, uint32_t stp) {
        if constexpr (SET::Q >= 9) {
            if (s.cn[5] != R(0)) return launch_kind<KIND, true>(b, t, s, st, stp);
        }
        launch_kind<KIND, false>(b, t, s, st, stp);
    }
    static int step(const StepBuffers &b, const void *tab, const void *sc, hipStream_t st,
                    uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        if (b.layout == kLocal)
            launch_step<kGatherScatter>(b, t, s, st, stp);
        else if (b.layout == kStreamed)
            launch_step<kNodeLocal>(b, t, s, st, stp);
        else
            launch_step<kPingPong>(b, t, s, st, stp);
        return hip_ok(hipGetLastError(), "step kernel launch");
    }
    static int init(void *dst, int layout, double *a_out, const double *rho, const double *u,
                    const void *tab, const void *sc, hipStream_t st, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_init2d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, dst,
                           layout, a_out, rho, u, t, s, stp);
        return hip_ok(hipGetLastError(), "init kernel launch");
    }
    static int observe(const void *pop, int layout, const double *a_cur, const double * /*invd*/,
                       double *rho, double *u, double *partial, const void *tab, const void *sc,
                       hipStream_t st) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_observe2d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st,
                           pop, layout, a_cur, rho, u, partial, t, s);
        return hip_ok(hipGetLastError(), "observe kernel launch");
    }
    static int exportp(const void *pop, int layout, double *out, const void *tab, const void *sc,
                       hipStream_t st) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_export2d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st, pop,
                           layout, out, t, s);
        return hip_ok(hipGetLastError(), "export kernel launch");
    }
    static int importp(void *dst, int layout, double *a_out, const double *in, const void *tab,
                       const void *sc, hipStream_t st, uint32_t stp) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        hipLaunchKernelGGL((k_import2d<SET, S>), dim3(blocks_for(s.nodes)), dim3(256), 0, st,
                           dst, layout, a_out, in, t, s, stp);
        return hip_ok(hipGetLastError(), "import kernel launch");
    }
    static int run_resident(const StepBuffers &b, const void *tab, const void *sc, hipStream_t st,
                            uint32_t step0, int nsteps) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        if (s.nodes > kResidentMaxNodes || (b.layout != kLocal && b.layout != kStreamed))
            return fail(LBM_E_INVALID, "resident stepping: in-place problems of at most 256 nodes");
        bool n5 = false;
        if constexpr (SET::Q >= 9) n5 = s.cn[5] != R(0);
        if (n5) {
            if constexpr (SET::Q >= 9)
                hipLaunchKernelGGL((k_run2d<SET, S, true>), dim3(1), dim3(256), 0, st, b, t, s,
                                   step0, nsteps);
        } else {
            hipLaunchKernelGGL((k_run2d<SET, S, false>), dim3(1), dim3(256), 0, st, b, t, s, step0,
                               nsteps);
        }
        return hip_ok(hipGetLastError(), "resident step kernel launch");
    }
    // Two steps per launch (k_pair2d). Bands: the fewest that give every CU
    // a workgroup, so that the rows recomputed at band edges stay few; a
    // forced band height (tests, tuning) may be anything >= 1.
    template <int KIND>
    static int pair_launch(const StepBuffers &b, const PairTable<R> &t, const StepScalars<R> &s,
                           hipStream_t st, uint32_t stp, int band_rows) {
        using TL = PairTile<SET, typename St<S>::T, KIND>;
        if constexpr (!TL::ok) {
            return fail(LBM_E_UNSUPPORTED, "two-step kernel: stencil too wide for the LDS ring");
        } else {
            const int nstrips = (s.nx + TL::BX - 1) / TL::BX;
            if (band_rows <= 0) {
                int dev = 0, cus = 256;
                if (hipGetDevice(&dev) == hipSuccess)
                    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
                const int bands = std::max(1, std::min(s.ny, (cus + nstrips - 1) / nstrips));
                band_rows = (s.ny + bands - 1) / bands;
                band_rows = (band_rows + TL::RR - 1) / TL::RR * TL::RR;
            }
            const int bands = (s.ny + band_rows - 1) / band_rows;
            const dim3 g((unsigned)(nstrips * bands)), bl(TL::NT);
            bool n5 = false;
            if constexpr (SET::Q >= 9) n5 = s.cn[5] != R(0);
#define LBM_PAIR(AL, STR, N5V)                                                                  \
    hipLaunchKernelGGL((k_pair2d<SET, S, AL, STR, N5V, KIND>), g, bl, 0, st, b, t, s, stp, \
                       band_rows)
            const bool al = s.nx % 64 == 0, str = s.stream_stores != 0;
            if (n5) {
                if constexpr (SET::Q >= 9) {
                    if (al && str) LBM_PAIR(true, true, true);
                    else if (al) LBM_PAIR(true, false, true);
                    else LBM_PAIR(false, false, true);
                }
            } else {
                if (al && str) LBM_PAIR(true, true, false);
                else if (al) LBM_PAIR(true, false, false);
                else LBM_PAIR(false, false, false);
            }
#undef LBM_PAIR
            return hip_ok(hipGetLastError(), "two-step kernel launch");
        }
    }
    // mode 1: alternating phases; mode 2: producer and consumer waves; mode
    // 3: two producer groups and consumer waves
    static int pair(const StepBuffers &b, const void *tab, const void *sc, hipStream_t st,
                    uint32_t stp, int band_rows, int mode) {
        const auto &t = *(const PairTable<R> *)tab;
        const auto &s = *(const StepScalars<R> *)sc;
        if (b.layout != kDirect || !b.pop_out)
            return fail(LBM_E_INVALID, "two-step kernel: needs two population copies");
        return mode == 3   ? pair_launch<kPairTwin>(b, t, s, st, stp, band_rows)
               : mode == 2 ? pair_launch<kPairSplit>(b, t, s, st, stp, band_rows)
                           : pair_launch<kPairAlternate>(b, t, s, st, stp, band_rows);
    }
    static constexpr Launch table{&step,    &init,         &observe, &exportp,
                                  &importp, &run_resident,
                                  PairTile<SET, typename St<S>::T, kPairAlternate>::ok ? &pair
                                                                                    : nullptr,
                                  PairTile<SET, typename St<S>::T, kPairTwin>::ok,
                                  pair_twin_default<SET, typename St<S>::T>()};
};

#define LBM_2D(SET)                                                           \
    {SET::ID, Storage::F64, &L2<SET, Storage::F64>::table},                   \
        {SET::ID, Storage::F32, &L2<SET, Storage::F32>::table},               \
        {SET::ID, Storage::F32RAW, &L2<SET, Storage::F32RAW>::table},         \
        {SET::ID, Storage::F16DEV, &L2<SET, Storage::F16DEV>::table}

// FP32 deviations collided in FP64 with stochastic rounding: the channel sets
#define LBM_2D_SR(SET) {SET::ID, Storage::F32SR, &L2<SET, Storage::F32SR>::table}

const Launch *find_launch_2d(int set_id, Storage st) {
    static const Entry entries[] = {
        LBM_2D(SetD2V17), LBM_2D(SetD2V37), LBM_2D(SetD2V16), LBM_2D(SetD2V33), LBM_2D(SetD2V32),
        LBM_2D_SR(SetD2V17), LBM_2D_SR(SetD2V37),
    };
    for (const auto &e : entries)
        if (e.id == set_id && e.s == st) return e.l;
    return nullptr;
}

}  // namespace lbm
