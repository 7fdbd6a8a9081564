// C ABI of the single-solve path: parameters (Section V of the paper), caller
// buffers, and the launch sequence of the fused step kernel.
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "lbm_internal.h"

namespace lbm {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t plane_of(int64_t nodes) { return (nodes + 63) / 64 * 64; }

size_t storage_bytes(int s) {
    switch (s) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        case LBM_F16DEV: return 2;
        case LBM_F32RAW: return 4;
        case LBM_F32SR: return 4;
        default: return 0;
    }
}

int64_t nodes_of(const lbm_problem_t &p) {
    return (int64_t)p.nx * p.ny * (p.dim == 3 ? p.nz : 1);
}

// wall elements per face: 2D y-walls have nx; a duct's y-faces nx*nz, z-faces nx*ny
int64_t face_elems(const lbm_problem_t &p) {
    if (p.dim == 2) return p.nx;
    return std::max<int64_t>((int64_t)p.nx * p.nz, (int64_t)p.nx * p.ny);
}

// One population array updated in place (AA pattern) when a copy is at most
// this size, so that the array can stay largely in the 256 MB last-level cache;
// two ping-pong copies above it (measured on MI355X with one step per launch:
// in place is ~7% faster for a 155 MB array, ping-pong ~10% faster for a
// 1.3 GB one).
constexpr size_t kInPlaceMaxBytes = size_t(512) << 20;

// 2D problems in FP32 deviations or FP64 whose set has the two-step kernel
// step ping-pong from this size per copy, two steps per launch. Measured on
// MI355X, us per step in place -> two steps per launch: D2V37 FP32 1024 x 256
// (39 MB) 12.2 -> 13.8, 2048 x 256 (78 MB) 22.2 -> 19.7, 2048 x 512 43.2 ->
// 39.2, 2048 x 1024 92.6 -> 67.0; D2V37 FP64 1024 x 256 24.2 -> 21.5, 2048 x
// 512 94.4 -> 74.5; D2V17 FP32 2048 x 512 20.8 -> 17.6. (FP32 raw storage
// lost, 43.7 -> 46.2; FP16 deviations and FP32SR keep single steps.)
constexpr size_t kPairMinBytes = size_t(64) << 20;

bool pair_by_default(const Dvm &d, const lbm_problem_t &p, size_t copy_bytes) {
    if (p.dim != 2 || copy_bytes < kPairMinBytes) return false;
    if (p.storage != LBM_F32 && p.storage != LBM_F64) return false;
    const int id = match_set(d);
    const Launch *La = id < 0 ? nullptr : find_launch(id, (Storage)p.storage);
    return La && La->pair;
}

struct Layout {
    size_t copy_bytes = 0;      // one copy of the populations
    bool in_place = true;
    size_t pop_bytes = 0;       // caller's population buffer: one or two copies
    size_t apart_bytes = 0;     // one copy of the wall partials
    size_t partial_bytes = 0;   // observation block partials
    size_t invd_bytes = 0;      // 1 / D(e) per face and position along it
    size_t off_a0 = 0, off_a1 = 0, off_invd = 0, off_partial = 0, off_out = 0, scratch_bytes = 0;
};

// positions along a face: a duct's y faces vary with z, its z faces with y
int64_t face_positions(const lbm_problem_t &p) {
    return p.dim == 3 ? std::max(p.ny, p.nz) : 1;
}

Layout layout_of(const Dvm &d, const lbm_problem_t &p) {
    Layout L;
    const int64_t nodes = nodes_of(p);
    L.copy_bytes = align_up((size_t)d.V * plane_of(nodes) * storage_bytes(p.storage));
    // Specular reflection (accommodation < 1) reads another node's leaving
    // population, which the in-place kernels overwrite in the same step: such
    // problems step ping-pong.
    L.in_place = p.accommodation == 1.0 &&
                 (p.layout == LBM_LAYOUT_IN_PLACE ||
                  (p.layout == LBM_LAYOUT_AUTO && L.copy_bytes <= kInPlaceMaxBytes &&
                   !pair_by_default(d, p, L.copy_bytes)));
    L.pop_bytes = L.in_place ? L.copy_bytes : 2 * L.copy_bytes;
    L.apart_bytes = align_up(sizeof(double) * 4 * std::max(1, d.halo) * face_elems(p));
    L.partial_bytes = align_up(sizeof(double) * 2 * observe_blocks(nodes));
    L.invd_bytes = align_up(sizeof(double) * 4 * face_positions(p));
    L.off_a0 = 0;
    L.off_a1 = L.apart_bytes;
    L.off_invd = 2 * L.apart_bytes;
    L.off_partial = L.off_invd + L.invd_bytes;
    L.off_out = L.off_partial + L.partial_bytes;
    L.scratch_bytes = L.off_out + align_up(2 * sizeof(double));
    return L;
}

}  // namespace

int match_set(const Dvm &d) {
    for (const auto &vs : velocity_sets()) {
        if (vs.dim != d.dim || vs.V != d.V || vs.nr != d.n_rest) continue;
        bool same = true;
        for (size_t q = 0; q < vs.ex.size() && same; ++q) {
            const int *e = &d.vel[3 * (d.n_rest + 2 * q)];
            same = e[0] == vs.ex[q] && e[1] == vs.ey[q] && e[2] == vs.ez[q];
        }
        if (same) return vs.id;
    }
    return -1;
}

namespace {

int validate(const Dvm &d, const lbm_problem_t &p) {
    if (p.dim != d.dim) return fail(LBM_E_INVALID, "problem dim differs from the DVM's");
    if (p.nx < 1 || p.ny < 1 || (p.dim == 3 && p.nz < 1)) return fail(LBM_E_INVALID, "sizes must be positive");
    int hn = 0;
    for (int v = 0; v < d.V; ++v) {
        hn = std::max(hn, std::abs(d.vel[3 * v + 1]));
        if (p.dim == 3) hn = std::max(hn, std::abs(d.vel[3 * v + 2]));
    }
    if (hn > kMaxWallRows) return fail(LBM_E_UNSUPPORTED, "wall-normal velocity components above 16");
    if (p.ny < hn || (p.dim == 3 && p.nz < hn))
        return fail(LBM_E_INVALID, "ny (and nz) must be at least the largest wall-normal |e|");
    if (p.hermite_order < 2 || p.hermite_order > (d.Q + 1) / 2)
        return fail(LBM_E_INVALID, "hermite order must satisfy 2 <= N <= (Q+1)/2");
    if (p.hermite_order > 5)
        return fail(LBM_E_UNSUPPORTED, "kernels implement Hermite orders up to 5");
    if (!(p.kn > 0)) return fail(LBM_E_INVALID, "kn must be positive");
    if (p.g_set && (p.g[1] != 0.0 || (p.dim == 3 && p.g[2] != 0.0)))
        return fail(LBM_E_INVALID, "the body force must be parallel to the walls (g.n = 0)");
    if (!p.g_set && !(std::isfinite(p.ma))) return fail(LBM_E_INVALID, "ma must be finite");
    if (!(p.rho0 > 0)) return fail(LBM_E_INVALID, "rho0 must be positive");
    if (storage_bytes(p.storage) == 0) return fail(LBM_E_INVALID, "unknown storage");
    if (p.layout != LBM_LAYOUT_AUTO && p.layout != LBM_LAYOUT_IN_PLACE &&
        p.layout != LBM_LAYOUT_PING_PONG)
        return fail(LBM_E_INVALID, "unknown population layout");
    if (!(p.accommodation >= 0.0 && p.accommodation <= 1.0))
        return fail(LBM_E_INVALID, "accommodation must lie in [0, 1]");
    if (p.accommodation != 1.0 && p.dim != 2)
        return fail(LBM_E_UNSUPPORTED, "accommodation below 1 is implemented for 2D channels");
    if (p.accommodation != 1.0 && p.layout == LBM_LAYOUT_IN_PLACE)
        return fail(LBM_E_UNSUPPORTED,
                    "accommodation below 1 steps ping-pong (specular partners belong to other nodes)");
    if (d.V / 2 > kMaxPairs) return fail(LBM_E_UNSUPPORTED, "velocity set too large for the kernel tables");
    // kernels index populations and nodes with 32-bit integers
    if ((double)d.V * (double)plane_of(nodes_of(p)) >= 4294967296.0)
        return fail(LBM_E_UNSUPPORTED, "problem too large: V x nodes must stay below 2^32");
    return LBM_OK;
}

void derive(const Dvm &d, const lbm_problem_t &p, lbm_params_t &o) {
    std::memset(&o, 0, sizeof(o));
    o.tau = p.kn * std::sqrt(2.0 / M_PI);   // Eq. nm.13 with tau = nu (Eq. nm.11)
    o.dt = 1.0 / (d.c * p.ny);              // xi dt = e dx, dx = l0 / ny
    o.omega = o.dt / (o.tau + 0.5 * o.dt);  // Eq. nm.8
    if (p.g_set) {
        for (int k = 0; k < 3; ++k) o.g[k] = p.g[k];
    } else {
        o.g[0] = 8.0 * o.tau * p.ma;         // NS centreline g l0^2 / (8 nu) = ma
    }
    o.u_c = o.g[0] != 0.0 ? o.g[0] / (8.0 * o.tau) : (p.ma != 0.0 ? p.ma : 1.0);
    o.mdot_scale = 1.0 / (4.0 * o.u_c * p.kn);  // Eq. pf.1
    o.V = d.V;
    o.halo = d.halo;
}

}  // namespace

struct Solver {
    Dvm dvm;
    lbm_problem_t prob{};
    lbm_params_t par{};
    Storage st = Storage::F64;
    const Launch *L = nullptr;
    void *pop = nullptr;            // current population array
    void *pop_other = nullptr;      // ping-pong: the other copy; in place: null
    bool in_place = true;
    int layout = kLocal;            // PopLayout of pop
    double *apart[2] = {nullptr, nullptr};
    double *partial = nullptr;
    double *out = nullptr;          // two doubles of observation results, then the error word
    int *err = nullptr;             // set by a kernel whose bounded wait gave up
    double *invd = nullptr;
    std::vector<double> invd_host;  // source of the asynchronous upload of invd
    int cur = 0;
    hipStream_t stream = nullptr;
    alignas(16) unsigned char tab[sizeof(PairTable<double>)];
    alignas(16) unsigned char sc[sizeof(StepScalars<double>)];
    int64_t nodes = 0;
    int64_t steps = 0;
    // Graph replay of step sequences (see run_graph): cached executable graphs
    // keyed by the starting configuration and the step count, the private
    // stream they are captured on, and the longest sequence per graph (0: off).
    struct Graph {
        void *pop;
        int cur, layout, len;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipStream_t capture = nullptr;
    int graph_steps = 0;
    bool graphs_allowed = true;     // false for solvers that may not own runtime memory
    // Most steps per one-workgroup resident launch (0: off; see lbm_run).
    int resident_steps = 0;
    // Two ping-pong steps per launch (Launch::pair) and its band height (0: auto).
    int pair_steps = 0;             // 0 off, else the lbm_solver_set_pair_steps mode (1-3)
    int pair_band_rows = 0;
    ~Solver() {
        if (!graphs.empty() || capture) (void)hipStreamSynchronize(stream);
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
        if (capture) (void)hipStreamDestroy(capture);
    }
};

// Step sequences of small problems are launch-bound (a few microseconds of
// host overhead per launch against well under a microsecond of kernel time):
// up to kGraphMaxSteps consecutive steps are captured once into a HIP graph
// and replayed with one launch. Only kernel launches are captured. The step
// kernels of every storage but FP16 deviations ignore the step counter (only
// stochastic rounding keys on it), so a replay is bit for bit the launches it
// recorded; FP16 runs step one launch at a time. Graphs are used for
// population copies up to kGraphMaxBytes, where launch latency dominates.
// Problems of at most kResidentMaxNodes nodes stepped in place (2D) run up to
// kResidentMaxSteps steps per launch in one workgroup (k_run2d), which also
// removes the device-side latency between dependent launches; FP16 included,
// since that kernel numbers the steps itself.
constexpr int kResidentMaxSteps = 4096;
constexpr int kGraphMaxSteps = 256;
constexpr size_t kGraphMaxBytes = size_t(16) << 20;
constexpr size_t kGraphCache = 8;

static bool resident_ok(const Solver &s) {
    return s.L->run_resident && s.in_place && s.prob.dim == 2 && s.nodes <= kResidentMaxNodes;
}

static bool pair_ok(const Solver &s) { return s.L->pair && !s.in_place; }

template <typename R>
static void fill_tables(const Dvm &d, const lbm_problem_t &p, const lbm_params_t &par, void *tab,
                        void *sc) {
    auto *t = new (tab) PairTable<R>();
    auto *s = new (sc) StepScalars<R>();
    std::memset(tab, 0, sizeof(PairTable<R>));
    std::memset(sc, 0, sizeof(StepScalars<R>));
    const double rho0 = p.rho0;
    auto shape = [&](int v) {
        double gx = 0;
        for (int k = 0; k < 3; ++k) gx += par.g[k] * d.c * d.vel[3 * v + k];
        return d.w[v] * (1.0 - 0.5 * par.dt * gx);
    };
    // half deviations are stored as 1024 d / (w rho0) (power of two: exact)
    const double enc = p.storage == LBM_F16DEV ? 1024.0 : 1.0;
    if (d.n_rest) {
        t->w0 = (R)d.w[0];
        t->wr00 = (R)(d.w[0] * rho0 / enc);
        t->inv_wr00 = (R)(enc / (d.w[0] * rho0));
        t->wrd0 = d.w[0] * rho0;
    }
    const int np = d.V / 2;
    for (int q = 0; q < np; ++q) {
        const int v = d.n_rest + 2 * q;
        t->w[q] = (R)d.w[v];
        t->wr0[q] = (R)(d.w[v] * rho0 / enc);
        t->inv_wr0[q] = (R)(enc / (d.w[v] * rho0));
        t->wrd[q] = d.w[v] * rho0;
    }
    s->rho0 = (R)rho0;
    s->rho0d = rho0;
    s->tau = (R)par.tau;
    s->omega = (R)par.omega;
    const double h = par.dt / (2.0 * par.tau);
    s->h = (R)h;
    s->inv1h = (R)(1.0 / (1.0 + h));
    for (int k = 0; k < 3; ++k) {
        s->g[k] = (R)par.g[k];
        s->half_dt_g[k] = (R)(0.5 * par.dt * par.g[k]);
    }
    double fact = 1.0;
    for (int k = 0; k < 6; ++k) {
        if (k > 0) fact *= k;
        s->cn[k] = k <= p.hermite_order ? (R)(1.0 / fact) : (R)0;
    }
    // D(e): emitted slots per element; uniform along each face of a channel
    double D[4] = {0, 0, 0, 0};
    for (int v = 0; v < d.V; ++v) {
        const int ey = d.vel[3 * v + 1];
        if (ey > 0) D[0] += ey * shape(v);
        if (ey < 0) D[1] += -ey * shape(v);
        if (d.dim == 3) {
            const int ez = d.vel[3 * v + 2];
            if (ez > 0) D[2] += ez * shape(v);
            if (ez < 0) D[3] += -ez * shape(v);
        }
    }
    for (int k = 0; k < 4; ++k) s->invD[k] = D[k] > 0 ? 1.0 / D[k] : 0.0;
    s->hgc = 0.5 * par.dt * par.g[0] * d.c;
    s->alpha = p.accommodation;
    s->specular = p.accommodation < 1.0 ? 1 : 0;
    // w rho0 of the populations that leave through each face from wall row r
    const bool dev_storage = deviation_storage((Storage)p.storage);
    for (int r = 0; r < kMaxWallRows; ++r) {
        double k[4] = {0, 0, 0, 0};
        for (int v = 0; v < d.V; ++v) {
            const int ey = d.vel[3 * v + 1], ez = d.vel[3 * v + 2];
            if (ey < -r) k[0] += d.w[v] * rho0;
            if (ey > r) k[1] += d.w[v] * rho0;
            if (ez < -r) k[2] += d.w[v] * rho0;
            if (ez > r) k[3] += d.w[v] * rho0;
        }
        for (int f = 0; f < 4; ++f) s->kA[f][r] = dev_storage ? k[f] : 0.0;
    }
    t->c = (R)d.c;
    s->nx = p.nx;
    s->ny = p.ny;
    s->nz = p.dim == 3 ? p.nz : 1;
    s->halo = d.halo;
    s->nodes = nodes_of(p);
    s->plane = plane_of(s->nodes);
    // aligned rows: whole 64-node blocks per row, at most 65536 rows (the
    // second dimension of their launch grid). Where the aligned kernels use
    // 32-bit buffer offsets (16-bit storage; channel stencils reaching
    // kBufferMinHalo columns) a population copy must stay below 2 GiB.
    const bool buffer = storage_bytes(p.storage) == 2 || (p.dim == 2 && d.halo >= kBufferMinHalo);
    s->aligned_rows = (p.nx % 64) == 0 && (int64_t)s->ny * s->nz <= 65536 &&
                      (!buffer || (double)d.V * (double)s->nodes * (double)storage_bytes(p.storage) <
                                      (double)(1u << 31));
    s->stream_stores = 2.0 * (double)d.V * (double)s->plane * (double)storage_bytes(p.storage) >
                       (double)(1u << 30);
}

// 1 / D(e) of a duct's wall elements, [face][position along the face]. A
// slot (x, alpha) whose virtual source x - e_alpha lies outside belongs to the
// face its segment crosses first going outward from x (ties to the y face) and
// to x's cell on that face; D(e) sums w (1 - dt/2 g.xi) over e's slots. It does
// not depend on x along the periodic direction, and y-face (z-face) elements
// only through z (y).
static void duct_invd(const Dvm &d, const lbm_problem_t &p, const lbm_params_t &par,
                      std::vector<double> &out) {
    const int ny = p.ny, nz = p.nz;
    const int64_t np = face_positions(p);
    std::vector<double> D(4 * np, 0.0);
    auto exit_time = [](int from, int v, int n) {
        const double plane = v > 0 ? (double)n - 0.5 : -0.5;
        return (plane - (double)from) / (double)v;
    };
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            if (j >= d.halo && j < ny - d.halo && k >= d.halo && k < nz - d.halo) continue;
            for (int v = 0; v < d.V; ++v) {
                const int *e = &d.vel[3 * v];
                const int js = j - e[1], ks = k - e[2];
                const bool oy = js < 0 || js >= ny, oz = ks < 0 || ks >= nz;
                if (!oy && !oz) continue;
                bool use_z = oz;
                if (oy && oz) use_z = exit_time(k, -e[2], nz) < exit_time(j, -e[1], ny);
                double gx = 0;
                for (int c = 0; c < 3; ++c) gx += par.g[c] * d.c * e[c];
                const double shape = d.w[v] * (1.0 - 0.5 * par.dt * gx);
                const int face = use_z ? (e[2] > 0 ? 2 : 3) : (e[1] > 0 ? 0 : 1);
                D[face * np + (use_z ? j : k)] += shape;
            }
        }
    out.assign(4 * np, 0.0);
    for (int64_t q = 0; q < 4 * np; ++q) out[q] = D[q] > 0 ? 1.0 / D[q] : 0.0;
}

// Validated parameters and kernel tables of one problem (used by the batch).
int problem_params(const Dvm &d, const lbm_problem_t &p, lbm_params_t &par, void *tab, void *sc,
                   bool f64) {
    int rc = validate(d, p);
    if (rc) return rc;
    derive(d, p, par);
    if (f64)
        fill_tables<double>(d, p, par, tab, sc);
    else
        fill_tables<float>(d, p, par, tab, sc);
    return LBM_OK;
}

static int sync_check(hipStream_t st) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("stream sync: ") + hipGetErrorString(e));
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" const char *lbm_last_error(void) { return g_err.c_str(); }

extern "C" int lbm_params(const lbm_dvm_t *dvm, const lbm_problem_t *prob, lbm_params_t *out) {
    if (!dvm || !prob || !out) return fail(LBM_E_INVALID, "lbm_params: null argument");
    const Dvm &d = *reinterpret_cast<const Dvm *>(dvm);
    int rc = validate(d, *prob);
    if (rc) return rc;
    derive(d, *prob, *out);
    return LBM_OK;
}

extern "C" int lbm_state_bytes(const lbm_dvm_t *dvm, const lbm_problem_t *prob, size_t *pop_bytes,
                               size_t *scratch_bytes) {
    if (!dvm || !prob) return fail(LBM_E_INVALID, "lbm_state_bytes: null argument");
    const Dvm &d = *reinterpret_cast<const Dvm *>(dvm);
    int rc = validate(d, *prob);
    if (rc) return rc;
    Layout L = layout_of(d, *prob);
    if (pop_bytes) *pop_bytes = L.pop_bytes;
    if (scratch_bytes) *scratch_bytes = L.scratch_bytes;
    return LBM_OK;
}

// A solver over the caller's population buffer and a scratch buffer (the
// caller's, or the library's static one). Graph replay (captured graphs own
// runtime memory) only when `graphs`.
int lbm::solver_create(const lbm_dvm_t *dvm, const lbm_problem_t *prob, void *pop_a,
                       void *scratch, size_t scratch_bytes, void *stream, bool graphs,
                       lbm_solver_t **out) {
    if (!out) return fail(LBM_E_INVALID, "lbm_solver_create: null output");
    *out = nullptr;
    if (!dvm || !prob || !pop_a || !scratch)
        return fail(LBM_E_INVALID, "lbm_solver_create: null argument");
    const Dvm &d = *reinterpret_cast<const Dvm *>(dvm);
    int rc = validate(d, *prob);
    if (rc) return rc;
    Layout L = layout_of(d, *prob);
    if (scratch_bytes < L.scratch_bytes) return fail(LBM_E_NO_MEMORY, "lbm_solver_create: scratch too small");
    for (void *ptr : {pop_a, scratch})
        if ((uintptr_t)ptr % kAlign) return fail(LBM_E_INVALID, "lbm_solver_create: buffers must be 256-byte aligned");
    const Storage st = (Storage)prob->storage;
    const int set_id = match_set(d);
    if (set_id < 0) return fail(LBM_E_UNSUPPORTED, "no kernel compiled for this velocity set");
    const Launch *La = find_launch(set_id, st);
    if (!La) return fail(LBM_E_UNSUPPORTED, "no kernel compiled for this velocity set / storage");
    auto *s = new Solver();
    s->dvm = d;
    s->prob = *prob;
    derive(d, *prob, s->par);
    s->st = st;
    s->L = La;
    s->in_place = L.in_place;
    s->pop = pop_a;
    s->pop_other = L.in_place ? nullptr : (void *)((unsigned char *)pop_a + L.copy_bytes);
    s->layout = L.in_place ? kLocal : kDirect;
    auto *base = (unsigned char *)scratch;
    s->apart[0] = (double *)(base + L.off_a0);
    s->apart[1] = (double *)(base + L.off_a1);
    s->invd = (double *)(base + L.off_invd);
    s->partial = (double *)(base + L.off_partial);
    s->out = (double *)(base + L.off_out);
    s->err = (int *)(base + L.off_out + 2 * sizeof(double));
    s->stream = (hipStream_t)stream;
    s->nodes = nodes_of(*prob);
    s->graph_steps =
        (graphs && !stochastic_storage(st) && L.copy_bytes <= kGraphMaxBytes) ? kGraphMaxSteps : 0;
    s->graphs_allowed = graphs;
    s->resident_steps = resident_ok(*s) ? kResidentMaxSteps : 0;
    // two steps per launch for ping-pong problems not stepped from graphs:
    // two producer groups and consumer waves (mode 3) where the kernel table
    // prefers them, else one producer group (mode 2). Measured on MI355X,
    // D2V37 FP32 4096 x 2048 (1.24 GB per copy): 230 us per step (mode 3) and
    // 269 us (mode 2) against 437 us for one launch per step. FP16 deviations
    // keep single steps: their step is bound by its arithmetic (252 against
    // 319 us); so do FP32SR's (FP64 collision).
    s->pair_steps = (pair_ok(*s) && s->graph_steps == 0 && !stochastic_storage(st))
                        ? (s->L->pair_twin_default ? 3 : 2)
                        : 0;
    if (st == Storage::F64 || st == Storage::F32SR)
        fill_tables<double>(d, *prob, s->par, s->tab, s->sc);
    else
        fill_tables<float>(d, *prob, s->par, s->tab, s->sc);
    // zero the wall partials so a run before init is well defined, and the
    // error word
    rc = launch_zero(scratch, L.off_partial, s->stream);
    if (rc == LBM_OK) rc = launch_zero(s->out, L.scratch_bytes - L.off_out, s->stream);
    if (rc) {
        delete s;
        return rc;
    }
    hipError_t e = hipSuccess;
    if (prob->dim == 3) {
        duct_invd(d, *prob, s->par, s->invd_host);
        e = hipMemcpyAsync(s->invd, s->invd_host.data(), sizeof(double) * s->invd_host.size(),
                           hipMemcpyHostToDevice, s->stream);
    }
    if (e != hipSuccess) {
        delete s;
        return fail(LBM_E_DEVICE, std::string("1/D(e) upload: ") + hipGetErrorString(e));
    }
    *out = reinterpret_cast<lbm_solver_t *>(s);
    return LBM_OK;
}

extern "C" int lbm_solver_create(const lbm_dvm_t *dvm, const lbm_problem_t *prob, void *pop_a,
                                 void *pop_b, void *scratch, size_t scratch_bytes, void *stream,
                                 lbm_solver_t **out) {
    (void)pop_b;  // pop_a holds both copies when the problem is stepped ping-pong
    return solver_create(dvm, prob, pop_a, scratch, scratch_bytes, stream, true, out);
}

extern "C" int lbm_solver_destroy(lbm_solver_t *h) {
    delete reinterpret_cast<Solver *>(h);
    return LBM_OK;
}

extern "C" int lbm_init_equilibrium(lbm_solver_t *h, const double *rho_dev, const double *u_dev) {
    if (!h) return fail(LBM_E_INVALID, "lbm_init_equilibrium: null handle");
    Solver &s = *reinterpret_cast<Solver *>(h);
    s.cur = 0;
    s.steps = 0;
    s.layout = s.in_place ? kLocal : kDirect;
    return s.L->init(s.pop, s.layout, s.apart[0], rho_dev, u_dev, s.tab, s.sc, s.stream,
                     0xFFFFFFFFu);
}

// One step launch on stream st from the solver's current configuration, which
// it then advances.
static int step_once(Solver &s, hipStream_t st) {
    StepBuffers b{s.pop, s.pop_other, s.layout, s.apart[s.cur], s.apart[1 - s.cur], s.invd};
    int rc = s.L->step(b, s.tab, s.sc, st, (uint32_t)s.steps);
    if (rc) return rc;
    s.cur ^= 1;
    if (s.in_place)
        s.layout = s.layout == kLocal ? kStreamed : kLocal;
    else
        std::swap(s.pop, s.pop_other);
    ++s.steps;
    return LBM_OK;
}

// The executable graph of `len` (even) steps from the current configuration:
// from the cache, or captured on the private stream (nothing runs during the
// capture) and instantiated. An even count returns every alternating buffer
// to where it started, so one graph serves every replay from this state.
static int graph_for(Solver &s, int len, hipGraphExec_t *exec) {
    for (auto &g : s.graphs)
        if (g.pop == s.pop && g.cur == s.cur && g.layout == s.layout && g.len == len) {
            *exec = g.exec;
            return LBM_OK;
        }
    hipError_t e = hipSuccess;
    if (!s.capture) e = hipStreamCreateWithFlags(&s.capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(s.capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    void *pop = s.pop, *other = s.pop_other;
    const int cur = s.cur, layout = s.layout;
    const int64_t steps = s.steps;
    int rc = LBM_OK;
    for (int k = 0; k < len && rc == LBM_OK; ++k) rc = step_once(s, s.capture);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s.capture, &graph);
    // back to the starting configuration: the captured launches have not run
    s.pop = pop;
    s.pop_other = other;
    s.cur = cur;
    s.layout = layout;
    s.steps = steps;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    if (s.graphs.size() >= kGraphCache) {
        e = hipStreamSynchronize(s.stream);   // the oldest may still be in flight
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(ex);
            return fail(LBM_E_DEVICE, std::string("stream sync: ") + hipGetErrorString(e));
        }
        (void)hipGraphExecDestroy(s.graphs.front().exec);
        s.graphs.erase(s.graphs.begin());
    }
    s.graphs.push_back({s.pop, s.cur, s.layout, len, ex});
    *exec = ex;
    return LBM_OK;
}

extern "C" int lbm_run(lbm_solver_t *h, int64_t nsteps) {
    if (!h || nsteps < 0) return fail(LBM_E_INVALID, "lbm_run: bad arguments");
    Solver &s = *reinterpret_cast<Solver *>(h);
    int64_t k = 0;
    while (k < nsteps) {
        const int64_t left = nsteps - k;
        if (s.resident_steps >= 2 && left >= 2) {
            const int len = (int)std::min<int64_t>(left, s.resident_steps);
            StepBuffers b{s.pop, s.pop_other, s.layout, s.apart[s.cur], s.apart[1 - s.cur], s.invd};
            int rc = s.L->run_resident(b, s.tab, s.sc, s.stream, (uint32_t)s.steps, len);
            if (rc) return rc;
            if (len & 1) {
                s.cur ^= 1;
                s.layout = s.layout == kLocal ? kStreamed : kLocal;
            }
            s.steps += len;
            k += len;
            continue;
        }
        if (s.pair_steps && left >= 2) {
            StepBuffers b{s.pop,  s.pop_other, s.layout, s.apart[s.cur], s.apart[1 - s.cur],
                          s.invd, s.err};
            int rc = s.L->pair(b, s.tab, s.sc, s.stream, (uint32_t)s.steps, s.pair_band_rows,
                               s.pair_steps);
            if (rc) return rc;
            s.cur ^= 1;
            std::swap(s.pop, s.pop_other);
            s.steps += 2;
            k += 2;
            continue;
        }
        if (s.graph_steps >= 2 && left >= 2) {
            const int len = (int)std::min<int64_t>(left & ~int64_t(1), s.graph_steps & ~1);
            hipGraphExec_t ex = nullptr;
            int rc = graph_for(s, len, &ex);
            if (rc) return rc;
            hipError_t e = hipGraphLaunch(ex, s.stream);
            if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
            s.steps += len;   // an even count: buffers and layout are where they started
            k += len;
            continue;
        }
        int rc = step_once(s, s.stream);
        if (rc) return rc;
        ++k;
    }
    return LBM_OK;
}

extern "C" int lbm_solver_set_resident_steps(lbm_solver_t *h, int max_steps) {
    if (!h || max_steps < 0) return fail(LBM_E_INVALID, "lbm_solver_set_resident_steps: bad arguments");
    Solver &s = *reinterpret_cast<Solver *>(h);
    if (max_steps > 0 && !resident_ok(s))
        return fail(LBM_E_UNSUPPORTED, "resident stepping: 2D in-place problems of at most 256 nodes");
    s.resident_steps = std::min(max_steps, 1 << 20);
    return LBM_OK;
}

extern "C" int lbm_solver_set_pair_steps(lbm_solver_t *h, int on, int band_rows) {
    if (!h || band_rows < 0 || on < 0 || on > 3)
        return fail(LBM_E_INVALID, "lbm_solver_set_pair_steps: bad arguments");
    Solver &s = *reinterpret_cast<Solver *>(h);
    if (on && !pair_ok(s))
        return fail(LBM_E_UNSUPPORTED,
                    "two steps per launch: 2D ping-pong problems of a set with a compiled kernel");
    if (on == 3 && !s.L->pair_twin)
        return fail(LBM_E_UNSUPPORTED,
                    "two steps per launch: the two producer groups' ring does not fit the LDS");
    s.pair_steps = on;
    s.pair_band_rows = band_rows;
    return LBM_OK;
}

extern "C" int lbm_solver_set_graph_steps(lbm_solver_t *h, int max_steps) {
    if (!h || max_steps < 0) return fail(LBM_E_INVALID, "lbm_solver_set_graph_steps: bad arguments");
    Solver &s = *reinterpret_cast<Solver *>(h);
    if (max_steps > 0 && stochastic_storage(s.st))
        return fail(LBM_E_UNSUPPORTED, "graph replay: stochastic rounding keys on the step");
    if (max_steps > 0 && !s.graphs_allowed)
        return fail(LBM_E_UNSUPPORTED, "graph replay: this solver allocates nothing (static scratch)");
    s.graph_steps = std::min(max_steps, 4096);
    return LBM_OK;
}

static int observe_impl(Solver &s, double *rho_dev, double *u_dev, double *mdot, double *mass) {
    int rc = s.L->observe(s.pop, s.layout, s.apart[s.cur], s.invd, rho_dev, u_dev, s.partial,
                          s.tab, s.sc, s.stream);
    if (rc) return rc;
    if (!mdot && !mass) return LBM_OK;
    rc = launch_finalize(s.partial, observe_blocks(s.nodes), s.out, s.stream);
    if (rc) return rc;
    double host[4];   // the two results, then the error word
    hipError_t e = hipMemcpyAsync(host, s.out, sizeof(host), hipMemcpyDeviceToHost, s.stream);
    if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("copy: ") + hipGetErrorString(e));
    rc = sync_check(s.stream);
    if (rc) return rc;
    int err = 0;
    std::memcpy(&err, &host[2], sizeof(err));
    if (err) return fail(LBM_E_DEVICE, "a two-step launch gave up waiting: the state is invalid");
    if (mdot) *mdot = s.par.mdot_scale * host[0] / (double)s.nodes;
    if (mass) *mass = host[1];
    return LBM_OK;
}

extern "C" int lbm_observe(lbm_solver_t *h, double *rho_dev, double *u_dev, double *mdot_host,
                           double *mass_host) {
    if (!h) return fail(LBM_E_INVALID, "lbm_observe: null handle");
    return observe_impl(*reinterpret_cast<Solver *>(h), rho_dev, u_dev, mdot_host, mass_host);
}

extern "C" int lbm_run_to_tol(lbm_solver_t *h, double tol, int check_every, int64_t max_steps,
                              int64_t *steps, double *mdot) {
    if (!h || !(tol > 0) || check_every < 1 || max_steps < 0)
        return fail(LBM_E_INVALID, "lbm_run_to_tol: bad arguments");
    Solver &s = *reinterpret_cast<Solver *>(h);
    double prev = 0.0, cur = 0.0;
    bool have_prev = false;
    int64_t done = 0;
    int rc = LBM_E_NOT_CONVERGED;
    while (done < max_steps) {
        const int64_t n = std::min<int64_t>(check_every, max_steps - done);
        int r = lbm_run(h, n);
        if (r) return r;
        done += n;
        r = observe_impl(s, nullptr, nullptr, &cur, nullptr);
        if (r) return r;
        if (!std::isfinite(cur)) return fail(LBM_E_DEVICE, "mass flow is not finite");
        if (have_prev && std::fabs(cur - prev) < tol * std::fabs(cur)) {
            rc = LBM_OK;
            break;
        }
        prev = cur;
        have_prev = true;
    }
    if (steps) *steps = done;
    if (mdot) *mdot = cur;
    if (rc) return fail(rc, "lbm_run_to_tol: step limit reached");
    return LBM_OK;
}

extern "C" int lbm_export_populations(lbm_solver_t *h, double *out_dev) {
    if (!h || !out_dev) return fail(LBM_E_INVALID, "lbm_export_populations: null argument");
    Solver &s = *reinterpret_cast<Solver *>(h);
    return s.L->exportp(s.pop, s.layout, out_dev, s.tab, s.sc, s.stream);
}

extern "C" int lbm_import_populations(lbm_solver_t *h, const double *in_dev) {
    if (!h || !in_dev) return fail(LBM_E_INVALID, "lbm_import_populations: null argument");
    Solver &s = *reinterpret_cast<Solver *>(h);
    s.cur = 0;  // the step counter is kept: a resumed run continues its numbering
    s.layout = s.in_place ? kLocal : kDirect;
    return s.L->importp(s.pop, s.layout, s.apart[0], in_dev, s.tab, s.sc, s.stream, 0xFFFFFFFEu);
}

extern "C" int lbm_solver_steps(const lbm_solver_t *h, int64_t *steps) {
    if (!h || !steps) return fail(LBM_E_INVALID, "lbm_solver_steps: null argument");
    *steps = reinterpret_cast<const Solver *>(h)->steps;
    return LBM_OK;
}
