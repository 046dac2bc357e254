// rsph_internal.h -- device-side data layout shared by the HIP kernels and the
// host side of librsph.so.  Not part of the C-ABI.
//
// Layout (all systems of a pool packed in one set of arrays):
//  * particles live in "slots"; each system owns a contiguous slot range that
//    starts on a multiple of 64, so a wavefront never spans two systems and the
//    per-wave table wave_sys[] gives the system of every lane;
//  * within a system's range particles are sorted by cell key, ties by the
//    caller's particle index (a deterministic, bit-exact order);
//  * FP64 state is structure-of-arrays; the inputs of the pair loops are packed
//    per particle into 4-wide records (float4 in the mixed form, double4 in the
//    FP64 form) so that one neighbour gather is one or two 16-byte loads;
//  * neighbour lists are stored per wavefront, transposed: entry k of lane l of
//    wave w is nbr[(w * kmax + k) * 64 + l], so the 64 lanes of a wave read 256
//    contiguous bytes at every step k.  An entry holds the neighbour's slot in
//    its low 26 bits and, in two bits per axis (x at bit 26, y at 28, z at 30),
//    the particle's cell minus the neighbour's stencil cell, plus one (0, 1 or
//    2): the mixed form rebuilds r_ij from the FP32 offsets in the cells and
//    these cell differences.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsph {

constexpr int kWave = 64;
constexpr int kBlock = 256;
// systems with at most this many force-pass blocks (65,536 slots at 4 lanes per
// particle) end their substeps inside the continuity pass
constexpr int64_t kFuseDtEntries = 1024;
constexpr int kKmax2 = 64;   // neighbour capacity per particle, 2D (20 on a lattice)
constexpr int kKmax3 = 192;  // 3D (80 on a lattice)
constexpr int kMaxCellsPerAxis = 512;  // a system's cell keys then stay below 2^27
constexpr int kMaxLanes = 16;  // lanes per particle slot in the pair passes (at most)
constexpr int kNbrIndexBits = 26;
constexpr uint32_t kNbrIndexMask = (1u << kNbrIndexBits) - 1u;
constexpr int64_t kMaxSlots = (int64_t)1 << kNbrIndexBits;  // slots of a pool (at most)

// method switches (mirror of the public RSPH_* flags)
constexpr uint32_t kNoPenalty = 1u;
constexpr uint32_t kNoShift = 2u;
constexpr uint32_t kNoDensitySummation = 4u;
constexpr uint32_t kGbarOwnPhaseAverage = 8u;
constexpr uint32_t kPenaltyR3 = 16u;
constexpr uint32_t kNoSurface = 32u;

// health bits (mirror of RSPH_HEALTH_*)
constexpr uint32_t kHealthNonFinite = 1u;
constexpr uint32_t kHealthDensity = 2u;
constexpr uint32_t kHealthNeighbours = 4u;
constexpr uint32_t kHealthCoincident = 8u;
constexpr uint32_t kHealthClose = 16u;  // two particles closer than 1e-3 dp (input check only)
constexpr uint32_t kHealthDtCollapse = 32u;  // acoustic step below 1e-12 of its no-flow value
constexpr int64_t kMaxCells = 2048LL * 2048LL;  // capacity of the three-phase scan

// fluid id of a wall particle (0 and 1 are the fluids k and l): it never moves,
// its velocity is the wall's, and a fluid particle sees it as the mirror of
// itself (the one-sided Riemann wall condition)
constexpr int kWall = 2;

// per-particle flag bits, rebuilt every advection step
constexpr uint8_t kFlagInterface = 1;  // has a neighbour of the other fluid
constexpr uint8_t kFlagNearInterface = 2;  // itself or a neighbour has kFlagInterface

// Per-system constants, device resident, read-only inside the kernels.
struct SysConst {
    int32_t dim;
    uint32_t flags;
    int32_t ncell[3];
    int32_t fuse_dt;  // 1: the continuity pass ends each substep itself (small systems)
    int64_t p_off;   // first slot
    int64_t p_n;     // particles
    int64_t c_off;   // first global cell
    int64_t ncells;
    double box[3];
    double half_box[3];
    double inv_cell[3];  // ncell / box
    double cell[3];      // box / ncell
    double h;
    double inv_h;
    double cut2;       // (2h)^2
    double w_alpha;    // kernel normalisation
    double w0;         // W(0)
    double dw_coef;    // -5 alpha / h
    double sigma0;     // lattice kernel sum (self included)
    double rho0[2];
    double eta[2];
    double c0;
    double inv_c0;
    double c0sq;
    double gamma;
    double xi;
    double alpha_h2;   // alpha h^2 of Eq. 14
    double cfl_ad;
    double cfl_ac;
    double dtad_visc[2];  // cfl_ad rho0 h^2 / eta (inf if eta = 0)
    double dtac_surf[2];  // cfl_ac sqrt(rho0 h^3 / (2 pi gamma)) (inf if gamma = 0)
    double grav[3];
    double coincident2;   // (1e-9 h)^2
    double close2;        // (1e-3 dp)^2
    double mphase[2];     // the mass of every particle of fluid k and of fluid l, when uniform
    double inv_c0sq;      // 1 / c0^2
};

// Advection-step state of a system (device resident; each change is made by
// one thread per system):
//   idle -> boundary (outer-step target not reached) -> substepping (after the
//   advection-step prologue) -> ended -> boundary/idle.  A system whose
//   substeps are ended by the separate substep pass goes through ending (the
//   substep that completes the advection step, its continuity pass still to
//   run) before ended.
constexpr int32_t kIdle = 0;
constexpr int32_t kBoundary = 1;
constexpr int32_t kSubstepping = 2;
constexpr int32_t kEnding = 3;
constexpr int32_t kEnded = 4;

// Per-system dynamic scalars, device resident.
struct SysDyn {
    double dt_ad;
    double tau;
    double t;
    double dt[2];                    // acoustic step of substep k at [k & 1]
    double vmax[2];                  // per fluid, of the last velocity update
    int32_t state;                   // kIdle ... kEnded
    int32_t stepping;                // 1 while the advection-step prologue runs for this system
    int32_t binned;                  // 1: xd holds the positions of the last binning, slot by slot
    int32_t displaced;               // 1: the key pass found a particle more than one cell from it
    long long n_displaced;           // advection steps whose binning found such a particle
    uint32_t health;
    int32_t ksub_max;                // most substeps in one advection step since the host last looked
    long long ksub;                  // substeps started in the current advection step
    long long n_sub;
    long long n_outer;
    long long target;                // advection steps to reach
    double dt_last;
    // the substep as its force pass found it (stored by the system's first
    // force block, read by the continuity pass that ends the substep)
    int32_t sub_state;
    uint32_t sub_health;
    long long sub_ksub;
    double sub_tau;
};

struct DevArrays {
    int64_t P;       // slots the kernels cover (multiple of 256; the arrays may hold more)
    int64_t C;       // global cells the kernels cover
    int32_t kmax;
    int32_t mode;    // 0 = step, 1 = evaluate rates only (no state update)
    int32_t dt_pass; // 1: some system's substeps are ended by the separate substep pass
    int32_t one_sys_waves;  // pool of one system: its 64-slot blocks (0 otherwise)
    // 1: every system's fluid masses are uniform per fluid, so the substep
    // passes gather two records per neighbour, {frozen position} and
    // {velocity, pressure}, and recover rho = rho0 + p / c0^2 and V = m / rho
    int32_t packed;
    // 1: some system holds wall particles (0: the substep passes leave out the
    // wall branches)
    int32_t walls;
    // 1: a large pool, whose substep passes check the system's state before
    // any slot load, so that a launch with nothing to do reads almost nothing
    int32_t state_first;
    int32_t pad_;
    // FP64 state, structure of arrays
    double* pos[3];
    double* vel[3];
    double* rho;
    double* drho;
    double* mass;
    int32_t* id;
    int32_t* phase;
    // snapshot taken by the key pass, moved back in sorted order by the rank pass
    double* pos2[3];
    double* vel2[3];
    double* rho2;
    double* drho2;
    double* mass2;
    int32_t* id2;
    int32_t* phase2;
    // binning
    uint32_t* key;
    int32_t* rank;
    int32_t* perm;  // caller-order slot of each sorted slot (read back for the binning check)
    int32_t* tmp;   // slots in arrival order within each cell
    int32_t* cell_cnt;
    int32_t* cell_start;  // C + 1
    int32_t* cell_sys;
    int32_t* scan_part;
    int32_t* wave_sys;
    // pair-loop inputs (float4 or double4 records)
    void* geo;     // frozen positions + tag
    void* vbuf[2]; // velocity records by substep parity; packed: [0] {v, p} as the substep
                   // starts, [1] {kicked v, p} (force writes [1], continuity writes [0])
    void* th[2];   // {rho, V, p, 0}, substep parity
    void* col;     // {grad C, 1/|grad C|}
    void* av;      // viscous acceleration
    // the shift pass's records (Eq. 14), written by the advection pass:
    // bm[0] {frozen offsets, V B entries}, bm[1] {V B entries} (3D), bs the
    // last V B entry, bt the particle's own term B_i sum_j W'_ij V_j r_ij / r
    void* bm[2];
    void* bs;
    void* bt;
    uint8_t* flags;
    uint32_t* nbr;
    int32_t* ncount;
    double* xd;      // frozen FP64 position per slot (D doubles, phase in the signs of x and y),
                     // read by the neighbour build and the density summation
    uint32_t* xq;    // 3D: fixed-point offsets from the cell corner (3 per slot, 31 bits and a
                     // phase bit each), read by the mixed form's density summation
    // rates written by an evaluation (FP64, slot order)
    double* r_acc;    // 3 * P
    double* r_accp;
    double* r_accs;
    double* r_accv;
    double* r_gradc;
    double* r_drho;   // P
    double* r_b;      // 9 * P
    double* r_dr;     // 3 * P
    double* r_sigma;  // P
    // observables partials
    double* obs_part;
    double* obs_out;
    // per-wave partial maxima of |v| (bit patterns), [2 w] fluid k, [2 w + 1] fluid l
    unsigned long long* vpart;
    // per launch group: 1 if some system did work (kernel timing)
    int32_t* work;
    int64_t work_cap;
    // system tables
    const SysConst* sc;
    SysDyn* sd;
    int32_t nsys;
};

// host-callable launchers (rsph_kernels.hip)
struct Launch {
    hipStream_t stream;
    int dim;
    int fp64;  // 1: FP64 pair loops, 0: mixed
};

// optional events recorded by the dispatch itself around one kernel
struct Ev {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

void launch_fill_i32(const Launch& L, int32_t* p, int64_t n, int32_t v);
void launch_empty(const Launch& L, Ev ev);
void launch_set_stepping(const Launch& L, const DevArrays& A, const int32_t* mask);
void launch_set_targets(const Launch& L, const DevArrays& A, const long long* targets);
void launch_reset_ksub_max(const Launch& L, const DevArrays& A);
void launch_bin(const Launch& L, const DevArrays& A, int64_t group);
void launch_neighbours(const Launch& L, const DevArrays& A, Ev ev);
int lanes_per_particle(int dim);
void launch_advection(const Launch& L, const DevArrays& A, Ev ev);
void launch_shift(const Launch& L, const DevArrays& A, Ev ev);
void launch_colour(const Launch& L, const DevArrays& A, Ev ev);
void launch_force(const Launch& L, const DevArrays& A, Ev ev);
void launch_dt_substep(const Launch& L, const DevArrays& A, int64_t group);
void launch_continuity(const Launch& L, const DevArrays& A, Ev ev, int64_t group);
void launch_observables(const Launch& L, const DevArrays& A);
// what the device-side particle load found: probe[0] bit 0 an invalid input,
// bit 1 a wall particle; probe[1 + f] and probe[3 + f] the smallest and the
// largest mass bits of fluid f (positive doubles order as their bits); the
// caller sets probe to {0, ~0, ~0, 0, 0} first
constexpr int kLoadProbeWords = 5;
void launch_load_particles(const Launch& L, const DevArrays& A, int64_t p_off, int64_t n, const double* pos,
                           const double* vel, const int32_t* phase, const double* mass, const double* rho,
                           const double* box, const double* rho0, double sigma0, unsigned long long* probe);
void launch_store_rates(const Launch& L, const DevArrays& A, int64_t p_off, int64_t n, double* acc, double* drho);

constexpr int kObsPart = 16;  // partial sums per wave and pass
constexpr int kObsOut = 32;   // reduced values per system

}  // namespace rsph
