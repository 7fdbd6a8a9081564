// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lbmdvm.h"

namespace lbm {

// ---------------------------------------------------------------------------
// velocity sets
// ---------------------------------------------------------------------------
struct Dvm {
    int dim = 2, Q = 0, V = 0, n_groups = 0;
    int n_rest = 0;                 // velocities with e = 0 (0 or 1), stored first
    int halo = 0;                   // max |e_i|
    double c = 0.0;
    std::vector<int32_t> vel;       // V * 3 (z = 0 in 2D); rest first, then pairs (e, -e)
    std::vector<double> w;          // V
};

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// ---------------------------------------------------------------------------
// kernel-side tables, passed by value as kernel arguments
// ---------------------------------------------------------------------------
constexpr int kMaxPairs = 64;       // up to V = 129
constexpr int kMaxWallRows = 16;    // largest wall-normal |e| with compiled kernels

// Per-velocity constants for a solve; velocity alpha = n_rest + 2 p (+e_p) or
// n_rest + 2 p + 1 (-e_p). The velocity components themselves are compile-time
// constants of the kernels.
template <typename R>
struct PairTable {
    R w[kMaxPairs];                 // pair weight
    R wr0[kMaxPairs];               // w * rho0 (F16DEV: w * rho0 / 1024)
    R inv_wr0[kMaxPairs];           // 1 / wr0 (deviation storage)
    double wrd[kMaxPairs];          // w * rho0 in double
    R w0, wr00, inv_wr00;           // rest velocity (if any)
    double wrd0;
    R c;                            // lattice speed
};

// Scalars of the collision and geometry.
template <typename R>
struct StepScalars {
    R rho0, tau, omega, h, inv1h;   // h = dt / (2 tau), inv1h = 1 / (1 + h)
    R g[3], half_dt_g[3];           // g and dt/2 g
    R cn[6];                        // 1/n! for the Hermite terms, 0 beyond N
    double rho0d;
    double invD[4];                 // 1 / D(e) per face (2D: uniform along a face)
    double hgc;                     // dt/2 * g_x * c: wall shape w (1 - hgc e_x)
    double kA[4][kMaxWallRows];     // per face and wall row r: sum of w rho0 over the
                                    // velocities leaving through the face from row r
                                    // (deviation storages; 0 otherwise)
    double alpha;                   // accommodation: diffuse fraction of the wall (2D)
    int specular;                   // alpha < 1: the rest is reflected specularly
    int nx, ny, nz, halo;
    int64_t plane;                  // nodes rounded up to whole 64-node blocks
    int aligned_rows;               // nx is a multiple of 64: a row starts a block
    int stream_stores;              // populations (both copies) above 1 GiB: streaming stores
    int64_t nodes;
};

enum class Storage : int {
    F64 = LBM_F64,
    F32 = LBM_F32,
    F16DEV = LBM_F16DEV,
    F32RAW = LBM_F32RAW,
    F32SR = LBM_F32SR
};

// Storages whose stored values are deviations from w rho0, and whose rounding
// is stochastic (keyed on node and step).
constexpr bool deviation_storage(Storage s) {
    return s == Storage::F32 || s == Storage::F16DEV || s == Storage::F32SR;
}
constexpr bool stochastic_storage(Storage s) { return s == Storage::F16DEV || s == Storage::F32SR; }

// Layouts of the population array of a solve.
//   kDirect   : node x holds its own post-collision populations, velocity alpha
//               in slot alpha (two arrays, ping-pong pull steps);
// and, for one array updated in place (the AA pattern):
//   kLocal    : node x holds its own post-collision populations, velocity alpha
//               in the slot of -alpha (after init, import and kStreamed steps);
//   kStreamed : slot alpha of node y holds the post-collision population that
//               streams into y along alpha from y - e_alpha; a population that
//               leaves through a wall stays at its node, in the slot of -alpha
//               (after kLocal steps).
// A step on a kLocal array gathers from and writes to the neighbours; a step on
// a kStreamed array reads and writes the node itself. Both read and write the
// same set of locations per node, so nodes never race.
enum PopLayout : int { kLocal = 0, kStreamed = 1, kDirect = 2 };

// Buffers of one solve (device pointers).
struct StepBuffers {
    void *pop;                      // the population array (ping-pong: the source)
    void *pop_out;                  // ping-pong: the destination; in place: unused
    int layout;                     // PopLayout of pop before the step
    const double *a_cur;            // wall-flux partials of the current state [face][halo][elements]
    double *a_next;                 // wall-flux partials written by the step
    const double *invd;             // 3D: 1 / D(e) per face and position along it
    int *err;                       // set by a kernel whose bounded wait gave up (or null)
};

// Launchers (instantiated in the .hip translation units).
struct Launch {
    int (*step)(const StepBuffers &, const void *tab, const void *sc, hipStream_t, uint32_t step);
    int (*init)(void *pop, int layout, double *a_out, const double *rho, const double *u,
                const void *tab, const void *sc, hipStream_t, uint32_t step);
    int (*observe)(const void *pop, int layout, const double *a_cur, const double *invd,
                   double *rho, double *u, double *partial, const void *tab, const void *sc,
                   hipStream_t);
    int (*exportp)(const void *pop, int layout, double *out, const void *tab, const void *sc,
                   hipStream_t);
    int (*importp)(void *pop, int layout, double *a_out, const double *in, const void *tab,
                   const void *sc, hipStream_t, uint32_t step);
    // nsteps in-place steps of a problem of at most kResidentMaxNodes nodes in
    // one workgroup launch (null where not compiled)
    int (*run_resident)(const StepBuffers &, const void *tab, const void *sc, hipStream_t,
                        uint32_t step0, int nsteps);
    // two ping-pong steps in one launch (kDirect pop -> kDirect pop_out; a_cur
    // -> a_next): the intermediate state stays on chip (null where not
    // compiled). band_rows = rows per workgroup band (0: chosen for the chip).
    int (*pair)(const StepBuffers &, const void *tab, const void *sc, hipStream_t, uint32_t step,
                int band_rows, int mode);
    // whether pair() has the two-producer-group schedule (mode 3), and
    // whether it is the default two-step schedule (else mode 2)
    bool pair_twin = false;
    bool pair_twin_default = false;
};

// Channel stencils reaching at least this far (max |e_i|, the set's halo) use
// raw buffer addressing in the aligned step kernels whatever the storage.
constexpr int kBufferMinHalo = 7;

// Largest problem (nodes) stepped by one workgroup over many steps per launch:
// one node per thread of a 256-thread workgroup. Measured on MI355X for nx = 1
// channels: 3.0 against 4.0 us per step (graph replay) for D2V17 FP64 and 4.4
// against 5.8 us for D2V37 FP32 up to 256 nodes; at 512 nodes, two nodes per
// thread, it falls behind (5.3 against 4.5 us, 7.0 against 5.9 us).
constexpr int64_t kResidentMaxNodes = 256;

// Velocity sets with compiled kernels (library velocity order).
struct VelSetInfo {
    std::string name;
    int id = 0, dim = 0, V = 0, nr = 0;
    std::vector<int> ex, ey, ez;    // +e of each pair
};
const std::vector<VelSetInfo> &velocity_sets();

// Compiled set matching a DVM's velocity list exactly, or -1.
int match_set(const Dvm &d);

// Returns nullptr when no kernel is compiled for this combination.
const Launch *find_launch(int set_id, Storage s);

// Zero `bytes` (a multiple of 4) of device memory at p with a kernel.
int launch_zero(void *p, size_t bytes, hipStream_t st);

// Sum of `n` doubles laid out as partials[n][2] into out[2] in a fixed order.
int launch_finalize(const double *partials, int n, double *out, hipStream_t st);

int observe_blocks(int64_t nodes);

// lbm_solver_create over any scratch buffer; graph replay only when `graphs`
// (captured graphs own runtime memory).
int solver_create(const lbm_dvm_t *dvm, const lbm_problem_t *prob, void *pop_a, void *scratch,
                  size_t scratch_bytes, void *stream, bool graphs, lbm_solver_t **out);

}  // namespace lbm
