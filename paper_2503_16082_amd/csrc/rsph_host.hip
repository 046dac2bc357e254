// rsph_host.hip -- host side of librsph.so: parameter validation, packed
// multi-system device layout, the dual-criteria step driver (section 3.3 of
// arXiv 2503.16082) with device-side time-step control, observables and the
// C-ABI declared in include/rsph.h.
//
// A standalone system is a pool holding one system, so every path below is the
// served path with a batch of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <mutex>
#include <vector>

#include "rsph.h"
#include "rsph_internal.h"

using namespace rsph;

namespace {

thread_local std::string g_last_error;

struct HipError {
    hipError_t e;
    const char* what;
};

#define HIPCHECK(expr)                                        \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) throw HipError{_e, #expr};      \
    } while (0)

struct StatusError {
    rsph_status s;
    std::string msg;
};

[[noreturn]] void fail(rsph_status s, const std::string& msg) { throw StatusError{s, msg}; }

// Wendland C2 normalisation and the lattice kernel sum (self included) of a
// perfect lattice of spacing dp: the reference number density of the
// normalised density summation.
double kernel_alpha(int dim, double h)
{
    return dim == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
}

double kernel_w(int dim, double h, double r)
{
    const double q = r / h;
    if (q >= 2.0) return 0.0;
    const double a = 1.0 - 0.5 * q;
    return kernel_alpha(dim, h) * a * a * a * a * (1.0 + 2.0 * q);
}

double lattice_sigma0(int dim, double h, double dp)
{
    const int reach = (int)std::ceil(2.0 * h / dp) + 1;
    double s = 0.0;
    for (int a = -reach; a <= reach; ++a)
        for (int b = -reach; b <= reach; ++b)
            for (int c = (dim == 3 ? -reach : 0); c <= (dim == 3 ? reach : 0); ++c)
                s += kernel_w(dim, h, dp * std::sqrt((double)(a * a + b * b + c * c)));
    return s;
}

struct TimedLaunch {
    int kind;
    int64_t group;  // launch group: did work if some system was active in it
    hipEvent_t start, stop;
};

}  // namespace

// One launch cycle captured as a graph: valid for its substep count and for
// the exact kernel arguments (array addresses and capacities) it was captured
// with.
struct CycleGraph {
    int64_t m = -1;
    DevArrays view{};
    hipGraphExec_t exec = nullptr;
};
constexpr size_t kGraphCache = 6;

struct rsph_pool {
    int dim = 2;
    int precision = RSPH_FP64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    bool standalone = false;
    std::vector<rsph_system*> systems;  // index == device table row
    DevArrays A{};
    int64_t P_cap = 0, C_cap = 0;
    int S_cap = 0;
    size_t bytes = 0;
    std::vector<void*> allocs;
    int32_t* d_mask = nullptr;
    long long* d_targets = nullptr;
    int32_t* work_dev = nullptr;
    int64_t m_pred = 8;  // substeps launched per cycle
    std::string err;
    // kernel timing
    bool timing = false;
    uint32_t timing_mask = 0;
    int64_t next_group = 0;
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> event_pool;
    int64_t t_launches[RSPH_KERNEL_COUNT] = {};
    double t_ms[RSPH_KERNEL_COUNT] = {};
    // launch cycles captured as HIP graphs, replayed while kernel timing is off
    bool graphs = true;
    std::vector<CycleGraph> cycle_graphs;
    // pinned host staging of particle uploads (hipHostMalloc), grown on demand
    char* stage = nullptr;
    size_t stage_bytes = 0;
    // pinned host copies of the per-system state and targets, grown on demand
    SysDyn* pin_dyn = nullptr;
    long long* pin_targets = nullptr;
    size_t pin_rows = 0;
};

struct rsph_system {
    rsph_pool* pool = nullptr;
    bool owns_pool = false;
    rsph_params prm{};
    SysConst sc{};
    int64_t n = 0;
    int64_t p_off = 0, p_cap = 0;
    int64_t c_off = 0, ncells = 0;
    int row = -1;
    bool has_particles = false;
    // every particle of a fluid has the same mass (SysConst::mphase)
    bool uniform_mass = true;
    // the system holds wall particles
    bool has_walls = true;
    bool faulted = false;
    bool rates_valid = false;
    // as of the host's last read of the system's device state
    long long seen_outer = 0;  // advection steps done
    long long seen_sub = 0;    // acoustic substeps done
    long long sps = 0;         // most substeps of one advection step lately (0: none seen yet)
    long long first_sps = 0;   // estimate for the first advection step, from the uploaded state
    double v0max[2] = {0.0, 0.0};  // largest uploaded |v| per fluid
    std::string err;
};

namespace {

Launch launch_of(const rsph_pool* P)
{
    return Launch{P->stream, P->dim, P->precision == RSPH_FP64 ? 1 : 0};
}

int kmax_of(int dim) { return dim == 2 ? kKmax2 : kKmax3; }

void validate_params(const rsph_params* p)
{
    if (!p) fail(RSPH_EINVAL, "params is NULL");
    if (p->dim != 2 && p->dim != 3) fail(RSPH_EINVAL, "dim must be 2 or 3");
    if (p->precision != RSPH_FP64 && p->precision != RSPH_MIXED)
        fail(RSPH_EINVAL, "precision must be RSPH_FP64 or RSPH_MIXED");
    const double vals[] = {p->dp, p->h_over_dp, p->rho0[0], p->rho0[1], p->eta[0], p->eta[1],
                           p->c0, p->gamma, p->xi, p->alpha_shift, p->cfl_ad, p->cfl_ac,
                           p->gravity[0], p->gravity[1], p->gravity[2], p->u_ref};
    for (double v : vals)
        if (!std::isfinite(v)) fail(RSPH_EINVAL, "parameters must be finite");
    if (!(p->dp > 0) || !(p->h_over_dp > 0)) fail(RSPH_EINVAL, "dp and h_over_dp must be > 0");
    if (!(p->rho0[0] > 0) || !(p->rho0[1] > 0)) fail(RSPH_EINVAL, "rho0 must be > 0");
    if (p->eta[0] < 0 || p->eta[1] < 0) fail(RSPH_EINVAL, "eta must be >= 0");
    if (p->c0 < 0) fail(RSPH_EINVAL, "c0 must be > 0, or 0 for the rule c0 = 10 U_max");
    if (p->u_ref < 0) fail(RSPH_EINVAL, "u_ref must be >= 0");
    if (p->gamma < 0) fail(RSPH_EINVAL, "gamma must be >= 0");
    if (!(p->cfl_ad > 0) || !(p->cfl_ac > 0)) fail(RSPH_EINVAL, "CFL factors must be > 0");
    const double h = p->h_over_dp * p->dp;
    for (int a = 0; a < p->dim; ++a) {
        if (!std::isfinite(p->box[a]) || !(p->box[a] > 0)) fail(RSPH_EINVAL, "box must be > 0");
        const double nc = std::floor(p->box[a] / (2.0 * h));
        if (nc < 3) fail(RSPH_EINVAL, "box must hold at least 3 cells of edge 2h per axis");
        if (nc > kMaxCellsPerAxis) fail(RSPH_EINVAL, "at most 512 cells of edge 2h per axis");
    }
}

SysConst make_const(const rsph_params& p)
{
    SysConst S{};
    S.dim = p.dim;
    S.flags = p.flags;
    const double h = p.h_over_dp * p.dp;
    S.h = h;
    S.inv_h = 1.0 / h;
    S.cut2 = (2.0 * h) * (2.0 * h);
    for (int a = 0; a < 3; ++a) {
        if (a < p.dim) {
            S.ncell[a] = (int32_t)std::floor(p.box[a] / (2.0 * h));
            S.box[a] = p.box[a];
        } else {
            S.ncell[a] = 1;
            S.box[a] = 1.0;
        }
        S.half_box[a] = 0.5 * S.box[a];
        S.inv_cell[a] = (double)S.ncell[a] / S.box[a];
        S.cell[a] = S.box[a] / (double)S.ncell[a];
        S.grav[a] = a < p.dim ? p.gravity[a] : 0.0;
    }
    S.ncells = (int64_t)S.ncell[0] * S.ncell[1] * S.ncell[2];
    S.w_alpha = kernel_alpha(p.dim, h);
    S.w0 = S.w_alpha;
    S.dw_coef = -5.0 * S.w_alpha / h;
    S.sigma0 = lattice_sigma0(p.dim, h, p.dp);
    for (int f = 0; f < 2; ++f) {
        S.rho0[f] = p.rho0[f];
        S.eta[f] = p.eta[f];
        S.dtad_visc[f] = p.eta[f] > 0 ? p.cfl_ad * (p.rho0[f] * h * h / p.eta[f]) : INFINITY;
        S.dtac_surf[f] = p.gamma > 0
                             ? p.cfl_ac * std::sqrt(p.rho0[f] * h * h * h / (2.0 * M_PI * p.gamma))
                             : INFINITY;
    }
    // c0 = 0 (the rule of section 2) is resolved by effective_c0 once the
    // particles are known; until then the anticipated speed alone sets it
    const double c0 = p.c0 > 0 ? p.c0 : 10.0 * p.u_ref;
    S.c0 = c0;
    S.inv_c0 = c0 > 0 ? 1.0 / c0 : 0.0;
    S.c0sq = c0 * c0;
    S.gamma = p.gamma;
    S.xi = p.xi >= 0 ? p.xi : 1.3 * std::fabs(std::log10(p.rho0[0] / p.rho0[1])) + 0.6;
    S.alpha_h2 = p.alpha_shift * h * h;
    S.cfl_ad = p.cfl_ad;
    S.cfl_ac = p.cfl_ac;
    S.coincident2 = (1e-9 * h) * (1e-9 * h);
    S.close2 = (1e-3 * p.dp) * (1e-3 * p.dp);
    S.inv_c0sq = c0 > 0 ? 1.0 / (c0 * c0) : 0.0;
    // the default masses (uniform per fluid); upload_particles checks given ones
    for (int f = 0; f < 2; ++f) S.mphase[f] = p.rho0[f] / S.sigma0;
    return S;
}

// Section 2 sets the artificial sound speed to ten times the largest
// anticipated flow speed.  With c0 = 0 in the parameters that speed is the
// larger of u_ref and the largest initial particle speed.
double effective_c0(const rsph_params& p, int64_t n, const double* vel)
{
    if (p.c0 > 0) return p.c0;
    double vmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double v2 = 0.0;
        for (int a = 0; a < p.dim; ++a) v2 += vel[i * p.dim + a] * vel[i * p.dim + a];
        vmax = std::max(vmax, std::sqrt(v2));
    }
    const double c0 = 10.0 * std::max(p.u_ref, vmax);
    if (!(c0 > 0) || !std::isfinite(c0))
        fail(RSPH_EINVAL, "c0 = 0 needs u_ref > 0 or a moving particle (c0 = 10 U_max)");
    return c0;
}

// Constants of a system whose particles are set now: the c0 = 0 rule resolved.
SysConst const_for_particles(const rsph_params& p, int64_t n, const double* vel)
{
    rsph_params q = p;
    q.c0 = effective_c0(p, n, vel);
    return make_const(q);
}

// Allocation plan of a pool: the same walk either allocates (P given) or only
// sums the bytes it would allocate, so budget checks are exact.
struct Alloc {
    rsph_pool* P;  // nullptr: count only
    size_t bytes = 0;
    template <typename T>
    T* take(size_t count)
    {
        const size_t b = std::max<size_t>(count, 1) * sizeof(T);
        bytes += b;
        if (!P) return nullptr;
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(RSPH_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
        }
        P->allocs.push_back(p);
        P->bytes += b;
        return (T*)p;
    }
};

void drop_graphs(rsph_pool* P)
{
    for (auto& g : P->cycle_graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    P->cycle_graphs.clear();
}

void free_arrays(rsph_pool* P)
{
    drop_graphs(P);
    for (void* p : P->allocs) (void)hipFree(p);
    P->allocs.clear();
    P->bytes = 0;
    P->A = DevArrays{};
    P->P_cap = P->C_cap = 0;
    P->S_cap = 0;
}

// Walks every device array of a pool with the capacities given (M: the pool's
// allocator, or a carver of the fixed scratch array).
template <typename Mem>
size_t plan_arrays(Mem& M, int dim, int precision, DevArrays& A, int32_t*& mask, long long*& targets,
                   int32_t*& work, int64_t Pc, int64_t Cc, int Sc)
{
    A = DevArrays{};
    const size_t r4 = precision == RSPH_FP64 ? 32 : 16;
    A.P = Pc;
    A.C = Cc;
    A.kmax = kmax_of(dim);
    for (int a = 0; a < 3; ++a) {
        A.pos[a] = M.template take<double>(Pc);
        A.vel[a] = M.template take<double>(Pc);
        A.pos2[a] = M.template take<double>(Pc);
        A.vel2[a] = M.template take<double>(Pc);
    }
    A.rho = M.template take<double>(Pc);
    A.drho = M.template take<double>(Pc);
    A.mass = M.template take<double>(Pc);
    A.id = M.template take<int32_t>(Pc);
    A.phase = M.template take<int32_t>(Pc);
    A.rho2 = M.template take<double>(Pc);
    A.drho2 = M.template take<double>(Pc);
    A.mass2 = M.template take<double>(Pc);
    A.id2 = M.template take<int32_t>(Pc);
    A.phase2 = M.template take<int32_t>(Pc);
    A.key = M.template take<uint32_t>(Pc);
    A.rank = M.template take<int32_t>(Pc);
    A.perm = M.template take<int32_t>(Pc);
    A.tmp = M.template take<int32_t>(Pc);
    A.cell_cnt = M.template take<int32_t>(Cc);
    A.cell_start = M.template take<int32_t>(Cc + 1);
    A.cell_sys = M.template take<int32_t>(Cc);
    A.scan_part = M.template take<int32_t>(2048);
    A.wave_sys = M.template take<int32_t>(Pc / kWave);
    A.geo = M.template take<char>(Pc * r4);
    for (int k = 0; k < 2; ++k) {
        A.vbuf[k] = M.template take<char>(Pc * r4);
        A.th[k] = M.template take<char>(Pc * r4);
        A.bm[k] = M.template take<char>(Pc * r4);
    }
    A.bs = M.template take<char>(Pc * (r4 / 4));
    A.bt = M.template take<char>(Pc * r4);
    A.col = M.template take<char>(Pc * r4);
    A.av = M.template take<char>(Pc * r4);
    A.flags = M.template take<uint8_t>(Pc);
    A.nbr = M.template take<uint32_t>(Pc * (size_t)A.kmax);
    A.ncount = M.template take<int32_t>(Pc);
    A.xd = M.template take<double>(Pc * (dim == 2 ? 2 : 4));
    A.xq = M.template take<uint32_t>(dim == 3 ? 3 * Pc : 1);
    A.r_acc = M.template take<double>(3 * Pc);
    A.r_accp = M.template take<double>(3 * Pc);
    A.r_accs = M.template take<double>(3 * Pc);
    A.r_accv = M.template take<double>(3 * Pc);
    A.r_gradc = M.template take<double>(3 * Pc);
    A.r_drho = M.template take<double>(Pc);
    A.r_b = M.template take<double>(9 * Pc);
    A.r_dr = M.template take<double>(3 * Pc);
    A.r_sigma = M.template take<double>(Pc);
    A.obs_part = M.template take<double>((Pc / kWave) * kObsPart);
    A.vpart = M.template take<unsigned long long>(2 * (Pc * kMaxLanes / kWave));
    A.obs_out = M.template take<double>((size_t)Sc * kObsOut);
    A.sc = M.template take<SysConst>(Sc);
    A.sd = M.template take<SysDyn>(Sc);
    mask = M.template take<int32_t>(Sc);
    targets = M.template take<long long>(Sc);
    A.work_cap = 1 << 16;
    A.work = nullptr;
    work = M.template take<int32_t>(A.work_cap);
    return M.bytes;
}

size_t arrays_bytes(const rsph_pool* P, int64_t Pc, int64_t Cc, int Sc)
{
    Alloc M{nullptr};
    DevArrays A;
    int32_t* m;
    long long* t;
    int32_t* w;
    return plan_arrays(M, P->dim, P->precision, A, m, t, w, Pc, Cc, Sc);
}

// Allocates every device array for the capacities given (contents undefined).
void alloc_arrays(rsph_pool* P, int64_t Pc, int64_t Cc, int Sc)
{
    Alloc M{P};
    plan_arrays(M, P->dim, P->precision, P->A, P->d_mask, P->d_targets, P->work_dev, Pc, Cc, Sc);
    // binning expects zero cell counts (each scan clears the counts it reads);
    // kernel timing expects clear per-launch-group work flags
    launch_fill_i32(launch_of(P), P->A.cell_cnt, Cc, 0);
    launch_fill_i32(launch_of(P), P->work_dev, P->A.work_cap, 0);
    P->P_cap = Pc;
    P->C_cap = Cc;
    P->S_cap = Sc;
}

struct Layout {
    std::vector<int64_t> p_off, p_cap, c_off;
    int64_t P = 0, C = 0;
};

Layout plan(const std::vector<rsph_system*>& sys, const rsph_system* extra)
{
    Layout L;
    auto add = [&](const rsph_system* s) {
        int64_t cap = (s->n + kWave - 1) / kWave * kWave;
        L.p_off.push_back(L.P);
        L.p_cap.push_back(cap);
        L.c_off.push_back(L.C);
        L.P += cap;
        L.C += s->sc.ncells;
    };
    for (auto* s : sys) add(s);
    if (extra) add(extra);
    L.P = std::max<int64_t>((L.P + kBlock - 1) / kBlock * kBlock, kBlock);
    L.C = std::max<int64_t>(L.C, 1);
    if (L.C > kMaxCells) fail(RSPH_EINVAL, "more than 2048*2048 cells in one pool");
    if (L.P > kMaxSlots) fail(RSPH_EINVAL, "too many particle slots (2^26 per pool)");
    return L;
}

// Re-packs the pool's persistent particle state after systems were added or
// removed: every member keeps its particles, t and counters; slot ranges,
// cell ranges and the device tables are rebuilt.
void repack(rsph_pool* P, const std::vector<rsph_system*>& members)
{
    const hipStream_t st = P->stream;
    Layout L = plan(members, nullptr);
    const int S = (int)members.size();
    // download the dynamic scalars of the current members
    std::vector<SysDyn> dyn_old(P->systems.size());
    if (!P->systems.empty() && P->A.sd) {
        HIPCHECK(hipMemcpyAsync(dyn_old.data(), P->A.sd, sizeof(SysDyn) * P->systems.size(),
                                hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
    }
    const bool grow = L.P > P->P_cap || L.C > P->C_cap || S > P->S_cap;
    DevArrays old = P->A;
    std::vector<void*> old_allocs;
    size_t old_bytes = P->bytes;
    if (grow) {
        const int64_t Pc = std::max<int64_t>(
            L.P, std::min<int64_t>(kMaxSlots / kBlock * kBlock, P->P_cap + P->P_cap / 2 / kBlock * kBlock));
        const int64_t Cc = std::max<int64_t>(L.C, P->C_cap + P->C_cap / 2);
        const int Sc = std::max(S, P->S_cap + P->S_cap / 2 + 1);
        int64_t Pg = P->standalone ? L.P : Pc;
        int64_t Cg = P->standalone ? L.C : Cc;
        int Sg = P->standalone ? S : Sc;
        if (P->budget && !P->standalone) {
            // a pool with a budget takes all of it when it first grows: launch
            // grids follow the slots in use, so unused capacity costs no time,
            // and later admissions seldom reallocate (which copies every
            // member).  Cells: one per 4 slots at least; system rows: 64.
            const int Sb = std::max(Sg, 64);
            auto cells_for = [&](int64_t p) { return std::max<int64_t>(Cg, p / 4); };
            auto fits = [&](int64_t p) { return arrays_bytes(P, p, cells_for(p), Sb) <= P->budget; };
            if (fits(Pg)) {
                const int64_t top = kMaxSlots / kBlock * kBlock;
                int64_t lo = Pg, hi = Pg;
                while (hi < top && fits(std::min(top, hi * 2))) hi = std::min(top, hi * 2);
                lo = hi;
                hi = std::min(top, hi * 2);
                // largest multiple of kBlock in [lo, hi] that fits
                while (hi - lo > kBlock) {
                    const int64_t mid = (lo + hi) / 2 / kBlock * kBlock;
                    if (mid <= lo) break;
                    if (fits(mid)) lo = mid;
                    else hi = mid;
                }
                if (hi > lo && fits(hi)) lo = hi;
                Pg = lo;
                Cg = cells_for(lo);
                Sg = Sb;
            }
        }
        if (P->budget && arrays_bytes(P, Pg, Cg, Sg) > P->budget) {
            // no head room for growth: exactly what the members need
            Pg = L.P;
            Cg = L.C;
            Sg = S;
        }
        if (P->budget && arrays_bytes(P, Pg, Cg, Sg) > P->budget)
            fail(RSPH_EBUSY, "pool HBM budget exhausted");
        old_allocs.swap(P->allocs);
        P->bytes = 0;
        int32_t* old_mask = P->d_mask;
        long long* old_targets = P->d_targets;
        int32_t* old_work = P->work_dev;
        const int64_t oP = P->P_cap, oC = P->C_cap;
        const int oS = P->S_cap;
        try {
            alloc_arrays(P, Pg, Cg, Sg);
        } catch (...) {
            for (void* p : P->allocs) (void)hipFree(p);
            P->allocs.swap(old_allocs);
            P->bytes = old_bytes;
            P->A = old;
            P->d_mask = old_mask;
            P->d_targets = old_targets;
            P->work_dev = old_work;
            P->P_cap = oP;
            P->C_cap = oC;
            P->S_cap = oS;
            throw;
        }
    }
    DevArrays& A = P->A;
    // the kernels cover the slots and cells in use, not the capacity
    A.P = L.P;
    A.C = L.C;
    // copy each member's persistent state from its old range into the
    // second buffer (new capacity, new offsets), then make that current; not
    // needed when no member moves (an admission that fits appends its system)
    bool moved = grow;
    for (int k = 0; k < S; ++k)
        if (members[k]->has_particles && members[k]->row >= 0 && L.p_off[k] != members[k]->p_off) moved = true;
    if (moved) {
        double** dst_d[] = {&A.pos2[0], &A.pos2[1], &A.pos2[2], &A.vel2[0], &A.vel2[1], &A.vel2[2],
                            &A.rho2, &A.drho2, &A.mass2};
        double* src_d[] = {old.pos[0], old.pos[1], old.pos[2], old.vel[0], old.vel[1], old.vel[2],
                           old.rho, old.drho, old.mass};
        int32_t** dst_i[] = {&A.id2, &A.phase2};
        int32_t* src_i[] = {old.id, old.phase};
        for (int k = 0; k < S; ++k) {
            rsph_system* s = members[k];
            if (!s->has_particles || s->row < 0) continue;
            for (int q = 0; q < 9; ++q)
                HIPCHECK(hipMemcpyAsync(*dst_d[q] + L.p_off[k], src_d[q] + s->p_off,
                                        sizeof(double) * s->n, hipMemcpyDeviceToDevice, st));
            for (int q = 0; q < 2; ++q)
                HIPCHECK(hipMemcpyAsync(*dst_i[q] + L.p_off[k], src_i[q] + s->p_off,
                                        sizeof(int32_t) * s->n, hipMemcpyDeviceToDevice, st));
        }
        for (int a = 0; a < 3; ++a) {
            std::swap(A.pos[a], A.pos2[a]);
            std::swap(A.vel[a], A.vel2[a]);
        }
        std::swap(A.rho, A.rho2);
        std::swap(A.drho, A.drho2);
        std::swap(A.mass, A.mass2);
        std::swap(A.id, A.id2);
        std::swap(A.phase, A.phase2);
    }
    // tables
    std::vector<SysConst> sc(S);
    std::vector<SysDyn> sd(S);
    std::vector<int32_t> wave(A.P / kWave, -1);
    std::vector<int32_t> csys(A.C, -1);
    const int lanes = lanes_per_particle(P->dim);
    A.dt_pass = 0;
    for (int k = 0; k < S; ++k) {
        rsph_system* s = members[k];
        SysDyn d{};
        if (s->row >= 0 && s->row < (int)dyn_old.size()) d = dyn_old[s->row];
        // the frozen positions of the last binning stay in the old slots:
        // the displacement check restarts at the system's next binning
        if (moved || L.p_off[k] != s->p_off) d.binned = 0;
        s->p_off = L.p_off[k];
        s->p_cap = L.p_cap[k];
        s->c_off = L.c_off[k];
        s->row = k;
        s->sc.p_off = s->p_off;
        s->sc.p_n = s->has_particles ? s->n : 0;
        s->sc.c_off = s->c_off;
        // per-block |v| partials of the force pass: small systems reduce them
        // inside every continuity block instead of in a pass of their own
        s->sc.fuse_dt = s->p_cap * lanes / kBlock <= kFuseDtEntries;
        if (!s->sc.fuse_dt) A.dt_pass = 1;
        sc[k] = s->sc;
        sd[k] = d;
        for (int64_t w = s->p_off / kWave; w < (s->p_off + s->p_cap) / kWave; ++w) wave[w] = k;
        for (int64_t c = s->c_off; c < s->c_off + s->ncells; ++c) csys[c] = k;
    }
    A.nsys = S;
    A.one_sys_waves = S == 1 ? (int32_t)(L.p_cap[0] / kWave) : 0;
    if (S) {
        HIPCHECK(hipMemcpyAsync((void*)A.sc, sc.data(), sizeof(SysConst) * S, hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(A.sd, sd.data(), sizeof(SysDyn) * S, hipMemcpyHostToDevice, st));
    }
    HIPCHECK(hipMemcpyAsync(A.wave_sys, wave.data(), sizeof(int32_t) * wave.size(), hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(A.cell_sys, csys.data(), sizeof(int32_t) * csys.size(), hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    for (void* p : old_allocs) (void)hipFree(p);
    P->systems = members;
    for (auto* s : members) s->rates_valid = false;
}

// ---- kernel timing ---------------------------------------------------------

hipEvent_t take_event(rsph_pool* P)
{
    if (!P->event_pool.empty()) {
        hipEvent_t e = P->event_pool.back();
        P->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    // timing-only events: no system-scope fence around the timed kernel
    HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
}

struct TimeScope {
    rsph_pool* P;
    int kind;
    int64_t group;
    bool on;
    Ev ev;
    TimeScope(rsph_pool* P_, int kind_, int64_t group_)
        : P(P_), kind(kind_), group(group_), on(P_->timing && ((P_->timing_mask >> kind_) & 1u))
    {
        if (!on) return;
        ev.start = take_event(P);
        ev.stop = take_event(P);
    }
    // events recorded around several launches (the binning sequence)
    void begin_range()
    {
        if (on) HIPCHECK(hipEventRecord(ev.start, P->stream));
    }
    void end_range()
    {
        if (on) HIPCHECK(hipEventRecord(ev.stop, P->stream));
    }
    ~TimeScope()
    {
        if (on) P->pending.push_back(TimedLaunch{kind, group, ev.start, ev.stop});
    }
};

// Folds recorded launches into the totals; launches of groups in which no
// system had work are dropped.
void collect_timing(rsph_pool* P)
{
    if (P->pending.empty() && P->next_group == 0) return;
    HIPCHECK(hipStreamSynchronize(P->stream));
    std::vector<int32_t> work(std::max<int64_t>(P->next_group, 1), 0);
    if (P->next_group > 0)
        HIPCHECK(hipMemcpy(work.data(), P->work_dev, sizeof(int32_t) * P->next_group, hipMemcpyDeviceToHost));
    for (auto& t : P->pending) {
        if (t.group < 0 || (t.group < P->next_group && work[t.group])) {
            float ms = 0.f;
            HIPCHECK(hipEventElapsedTime(&ms, t.start, t.stop));
            P->t_ms[t.kind] += ms;
            P->t_launches[t.kind] += 1;
        }
        P->event_pool.push_back(t.start);
        P->event_pool.push_back(t.stop);
    }
    P->pending.clear();
    if (P->next_group > 0) launch_fill_i32(launch_of(P), P->work_dev, P->next_group, 0);
    P->next_group = 0;
}

// ---- driver ----------------------------------------------------------------

void set_mask(rsph_pool* P, const std::vector<int32_t>& mask)
{
    HIPCHECK(hipStreamSynchronize(P->stream));
    HIPCHECK(hipMemcpy(P->d_mask, mask.data(), sizeof(int32_t) * mask.size(), hipMemcpyHostToDevice));
    launch_set_stepping(launch_of(P), P->A, P->d_mask);
}

DevArrays kernel_view(rsph_pool* P)
{
    DevArrays A = P->A;
    A.work = P->timing ? P->work_dev : nullptr;
    // the packed substep passes (8.4M particles in 3D: force 2.81 -> 2.55 ms,
    // continuity 2.43 -> 1.73 ms; 40,000 in 2D: 0.6 % more particle-steps/s,
    // a 256-system pool 1.8 %) whenever every system's fluid masses are uniform
    A.packed = 1;
    A.walls = 0;
    // an idle substep launch over 8.4M slots fetched 0.5 GB of slot-only loads
    // and took 0.26 ms; small pools keep the loads ahead of the state check,
    // which shortens their latency-bound launches
    A.state_first = P->A.P >= ((int64_t)1 << 20) ? 1 : 0;
    for (const rsph_system* s : P->systems) {
        if (s && !s->uniform_mass) A.packed = 0;
        if (s && s->has_walls) A.walls = 1;
    }
    return A;
}

// binning and neighbour lists: in step mode for the systems that the key pass
// puts at the start of an advection step, otherwise for the systems whose
// stepping flag the caller set
void rebuild(rsph_pool* P, int mode, int64_t group)
{
    const Launch L = launch_of(P);
    DevArrays A = kernel_view(P);
    A.mode = mode;
    {
        TimeScope t(P, RSPH_KERNEL_BIN, group);
        t.begin_range();
        launch_bin(L, A, group);
        t.end_range();
    }
    TimeScope t(P, RSPH_KERNEL_NEIGHBOURS, group);
    launch_neighbours(L, A, t.ev);
}

// pinned host rows for the per-system state and targets (no copy may be in
// flight from or to them: every stepping call ends with a stream sync)
void ensure_pinned_rows(rsph_pool* P, size_t rows)
{
    if (rows <= P->pin_rows) return;
    if (P->pin_dyn) HIPCHECK(hipHostFree(P->pin_dyn));
    if (P->pin_targets) HIPCHECK(hipHostFree(P->pin_targets));
    P->pin_dyn = nullptr;
    P->pin_targets = nullptr;
    P->pin_rows = 0;
    const size_t n = std::max<size_t>(rows, 64);
    HIPCHECK(hipHostMalloc((void**)&P->pin_dyn, sizeof(SysDyn) * n, hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void**)&P->pin_targets, sizeof(long long) * n, hipHostMallocDefault));
    P->pin_rows = n;
}

std::vector<SysDyn> read_dyn(rsph_pool* P)
{
    std::vector<SysDyn> d(P->systems.size());
    if (!d.empty()) {
        ensure_pinned_rows(P, d.size());
        HIPCHECK(hipMemcpyAsync(P->pin_dyn, P->A.sd, sizeof(SysDyn) * d.size(), hipMemcpyDeviceToHost, P->stream));
    }
    HIPCHECK(hipStreamSynchronize(P->stream));
    if (!d.empty()) std::memcpy(d.data(), P->pin_dyn, sizeof(SysDyn) * d.size());
    return d;
}

constexpr uint32_t kFaultBits =
    kHealthNonFinite | kHealthDensity | kHealthNeighbours | kHealthCoincident | kHealthDtCollapse;
constexpr int64_t kMaxSubsteps = 1000000;  // per advection step

// m acoustic substeps for the systems inside an advection step (the others
// exit at once)
void launch_substeps_eager(rsph_pool* P, int64_t m)
{
    const Launch L = launch_of(P);
    if (P->timing && P->next_group + m > P->A.work_cap) collect_timing(P);
    DevArrays A = kernel_view(P);
    A.mode = 0;
    for (int64_t q = 0; q < m; ++q) {
        const int64_t g = P->next_group++;
        {
            TimeScope t(P, RSPH_KERNEL_COLOUR, g);
            launch_colour(L, A, t.ev);
        }
        {
            TimeScope t(P, RSPH_KERNEL_FORCE, g);
            launch_force(L, A, t.ev);
        }
        if (A.dt_pass) launch_dt_substep(L, A, g);
        {
            TimeScope t(P, RSPH_KERNEL_CONTINUITY, g);
            launch_continuity(L, A, t.ev, g);
        }
    }
}

// One launch cycle: the advection-step prologue for systems at a boundary,
// then m acoustic substeps for systems inside an advection step.  Every kernel
// checks its system's state on the device, so no host synchronisation is
// needed between cycles.
void launch_cycle_eager(rsph_pool* P, int64_t m)
{
    const Launch L = launch_of(P);
    if (P->timing && P->next_group + m + 1 > P->A.work_cap) collect_timing(P);
    DevArrays A = kernel_view(P);
    A.mode = 0;
    const int64_t g0 = P->next_group++;
    rebuild(P, 0, g0);
    {
        TimeScope t(P, RSPH_KERNEL_ADVECTION, g0);
        launch_advection(L, A, t.ev);
    }
    {
        TimeScope t(P, RSPH_KERNEL_SHIFT, g0);
        launch_shift(L, A, t.ev);
    }
    launch_substeps_eager(P, m);
}

// A launch cycle, replayed from a captured graph unless kernel timing is on
// (timed launches carry their own events) or graphs are switched off.  The
// cycle holds kernel launches only, so its graph has kernel nodes only.
void launch_cycle(rsph_pool* P, int64_t m)
{
    if (P->timing || !P->graphs) {
        launch_cycle_eager(P, m);
        return;
    }
    const DevArrays A = kernel_view(P);
    CycleGraph* hit = nullptr;
    for (auto& g : P->cycle_graphs)
        if (g.m == m && std::memcmp(&g.view, &A, sizeof A) == 0) hit = &g;
    if (!hit) {
        if (P->cycle_graphs.size() >= kGraphCache) {
            (void)hipGraphExecDestroy(P->cycle_graphs.front().exec);
            P->cycle_graphs.erase(P->cycle_graphs.begin());
        }
        const int64_t group0 = P->next_group;
        hipGraph_t graph = nullptr;
        HIPCHECK(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
        try {
            launch_cycle_eager(P, m);
        } catch (...) {
            (void)hipStreamEndCapture(P->stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HIPCHECK(hipStreamEndCapture(P->stream, &graph));
        P->next_group = group0;
        hipGraphExec_t exec = nullptr;
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHECK(e);
        P->cycle_graphs.push_back(CycleGraph{m, A, exec});
        hit = &P->cycle_graphs.back();
    }
    HIPCHECK(hipGraphLaunch(hit->exec, P->stream));
}

// Substeps per launch cycle for the advection steps still to go (left[row]):
// the system with the most substeps to go is spread over as many cycles as
// the system with the most advection steps to go needs (a system takes at most
// one advection step per cycle).  A system's substeps per step are those of
// its recent steps; a system without any yet counts as the most of the others.
int64_t plan_substeps(const rsph_pool* P, const std::vector<long long>& left)
{
    double work = 0.0;
    long long steps = 0;
    for (size_t r = 0; r < left.size(); ++r) {
        if (left[r] <= 0 || P->systems[r]->faulted) continue;
        const long long sps = P->systems[r]->sps > 0 ? P->systems[r]->sps : P->m_pred;
        work = std::max(work, (double)left[r] * (double)sps);
        steps = std::max(steps, left[r]);
    }
    if (steps == 0) return P->m_pred;
    return std::min<int64_t>(4096, std::max<int64_t>(1, (int64_t)std::ceil(work / (double)steps)));
}

// Advances every system of the pool to its device-side target (left[row]
// advection steps to go).  Returns the OR of the health bits.  Cycles are
// launched in batches with one stream synchronisation after each; the
// substeps per cycle follow the systems' recent substeps per advection step
// (a step that needs more simply continues in the next cycle).  A system's
// first advection step does not count there: started from rest, it is bounded
// by the viscous criterion alone and can need many times the substeps of the
// steps after it.  When every system that still has work is only finishing
// its last advection step, the rest of that step is launched as substeps
// alone, as many as the longest of them still needs at its current acoustic
// step (a later batch adds more if the acoustic step shrinks).
uint32_t run_to_targets(rsph_pool* P, std::vector<long long> left)
{
    int64_t cycles = 1;
    for (long long l : left) cycles = std::max<int64_t>(cycles, l);
    int64_t batch = 4;
    int64_t m = plan_substeps(P, left);
    int64_t finish = 0;  // substeps alone, instead of cycles
    for (;;) {
        if (finish > 0) {
            launch_substeps_eager(P, finish);
        } else {
            const int64_t c = std::min(cycles, batch);
            for (int64_t k = 0; k < c; ++k) launch_cycle(P, m);
        }
        std::vector<SysDyn> d = read_dyn(P);
        uint32_t health = 0;
        int64_t remaining = 0;
        bool pending = false, new_steps = false;
        int64_t m_seen = 0, rest = 0;
        int32_t ksub_max = 0;
        for (size_t s = 0; s < d.size(); ++s) {
            rsph_system* sys = P->systems[s];
            health |= d[s].health;
            ksub_max = std::max(ksub_max, d[s].ksub_max);
            const long long l = d[s].target - d[s].n_outer;
            const bool inside = d[s].state == kSubstepping;
            const bool settled = sys->seen_outer >= 1;
            sys->seen_outer = d[s].n_outer;
            sys->seen_sub = d[s].n_sub;
            if (settled && d[s].ksub_max > 0) sys->sps = d[s].ksub_max;
            left[s] = std::max(l, 0LL);
            if (d[s].health & kFaultBits) {
                left[s] = 0;
                continue;
            }
            if (l > 0 || inside) pending = true;
            if (l > 1 || (l == 1 && !inside)) new_steps = true;
            remaining = std::max<int64_t>(remaining, l);
            if (settled) m_seen = std::max<int64_t>(m_seen, d[s].ksub_max);
            if (d[s].ksub > kMaxSubsteps) fail(RSPH_ENUMERIC, "more than 1e6 acoustic substeps in one advection step");
            if (inside && l == 1) {
                const double dt = d[s].dt[d[s].ksub & 1];
                const double r = dt > 0.0 ? std::ceil((d[s].dt_ad - d[s].tau) / dt) : (double)m;
                rest = std::max<int64_t>(rest, (int64_t)std::min(std::max(r, 1.0), 4096.0));
            }
        }
        if (m_seen > 0) P->m_pred = std::min<int64_t>(4096, m_seen);
        if (ksub_max > 0) launch_reset_ksub_max(launch_of(P), P->A);
        // faulted systems stay idle on the device; the others run to their targets
        if (!pending) return health;
        finish = new_steps ? 0 : rest;
        m = plan_substeps(P, left);
        cycles = std::max<int64_t>(remaining, 1);
        batch = std::min<int64_t>(batch * 2, 64);
    }
}

// new targets, copied in stream order (the pinned rows are free: the last
// stepping call ended with a stream sync)
void set_targets(rsph_pool* P, const std::vector<long long>& targets)
{
    if (targets.empty()) return;
    ensure_pinned_rows(P, targets.size());
    std::memcpy(P->pin_targets, targets.data(), sizeof(long long) * targets.size());
    HIPCHECK(hipMemcpyAsync(P->d_targets, P->pin_targets, sizeof(long long) * targets.size(),
                            hipMemcpyHostToDevice, P->stream));
    launch_set_targets(launch_of(P), P->A, P->d_targets);
}

template <typename F>
rsph_status guarded(std::string* err, F&& f)
{
    try {
        f();
        return RSPH_OK;
    } catch (const StatusError& e) {
        if (err) *err = e.msg;
        g_last_error = e.msg;
        return e.s;
    } catch (const HipError& e) {
        std::string m = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what;
        if (err) *err = m;
        g_last_error = m;
        return RSPH_EDEVICE;
    } catch (const std::bad_alloc&) {
        if (err) *err = "host allocation failed";
        g_last_error = "host allocation failed";
        return RSPH_ENOMEM;
    } catch (...) {
        if (err) *err = "unexpected error";
        g_last_error = "unexpected error";
        return RSPH_EDEVICE;
    }
}

void validate_particles(const rsph_params& p, int64_t n, const double* pos, const double* vel,
                        const int32_t* phase, const double* mass, const double* rho)
{
    if (n < 1) fail(RSPH_EINVAL, "n must be >= 1");
    if (n > kMaxSlots) fail(RSPH_EINVAL, "too many particles (2^26 per pool)");
    if (!pos || !vel || !phase) fail(RSPH_EINVAL, "pos, vel and phase are required");
    const int d = p.dim;
    for (int64_t i = 0; i < n * d; ++i)
        if (!std::isfinite(pos[i]) || !std::isfinite(vel[i])) fail(RSPH_EINVAL, "non-finite position or velocity");
    for (int64_t i = 0; i < n; ++i)
        if (phase[i] != 0 && phase[i] != 1 && phase[i] != kWall)
            fail(RSPH_EINVAL, "phase must be 0, 1 (the fluids) or 2 (a wall particle)");
    if (mass)
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(mass[i]) || !(mass[i] > 0)) fail(RSPH_EINVAL, "mass must be finite and > 0");
    if (rho)
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(rho[i]) || !(rho[i] > 0)) fail(RSPH_EINVAL, "rho must be finite and > 0");
}

// The per-fluid masses of the particles given (NULL: the defaults): a fluid
// whose particles all have one mass keeps it in the constants, which lets the
// substep passes recover a neighbour's volume from its density alone; any
// other mix of masses sends the pool through the passes that gather the volume.
void set_fluid_masses(rsph_system* s, int64_t n, const int32_t* phase, const double* mass)
{
    s->has_walls = std::find(phase, phase + n, kWall) != phase + n;
    s->uniform_mass = true;
    if (!mass) return;
    bool seen[2] = {false, false};
    for (int64_t i = 0; i < n; ++i) {
        if (phase[i] == kWall) continue;  // the substep passes never read a wall's mass
        const int f = phase[i];
        if (!seen[f]) {
            seen[f] = true;
            s->sc.mphase[f] = mass[i];
        } else if (mass[i] != s->sc.mphase[f]) {
            s->uniform_mass = false;
            return;
        }
    }
}

// Uploads particles into the system's (already planned) slot range.
void upload_particles(rsph_system* s, const double* pos, const double* vel, const int32_t* phase,
                      const double* mass, const double* rho)
{
    rsph_pool* P = s->pool;
    HIPCHECK(hipStreamSynchronize(P->stream));
    const int64_t n = s->n;
    const int d = s->prm.dim;
    // the fields are staged in pinned host memory, a bounded chunk of
    // particles at a time, and each chunk is copied with one stream sync
    constexpr int64_t kChunk = 1 << 19;
    const int64_t cn = std::min<int64_t>(n, kChunk);
    const size_t need = (sizeof(double) * 9 + sizeof(int32_t) * 2) * (size_t)cn;
    if (need > P->stage_bytes) {
        if (P->stage) HIPCHECK(hipHostFree(P->stage));
        P->stage = nullptr;
        P->stage_bytes = 0;
        HIPCHECK(hipHostMalloc((void**)&P->stage, need, hipHostMallocDefault));
        P->stage_bytes = need;
    }
    double* f = (double*)P->stage;
    int32_t* ib = (int32_t*)(f + 9 * cn);
    s->v0max[0] = s->v0max[1] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (phase[i] == kWall) continue;  // a wall's speed is not the fluids'
        double v2 = 0.0;
        for (int a = 0; a < d; ++a) v2 += vel[i * d + a] * vel[i * d + a];
        double& vm = s->v0max[phase[i] & 1];
        vm = std::max(vm, std::sqrt(v2));
    }
    double* dst[9] = {P->A.pos[0], P->A.pos[1], P->A.pos[2], P->A.vel[0], P->A.vel[1], P->A.vel[2],
                      P->A.mass, P->A.rho, P->A.drho};
    for (int64_t i0 = 0; i0 < n; i0 += cn) {
        const int64_t m = std::min(cn, n - i0);
        for (int64_t k = 0; k < m; ++k) {
            const int64_t i = i0 + k;
            for (int a = 0; a < 3; ++a) {
                double q = a < d ? pos[i * d + a] : 0.0;
                if (a < d) {
                    const double L = s->prm.box[a];
                    q = q - L * std::floor(q / L);
                    if (q >= L) q -= L;
                }
                f[a * cn + k] = q;
                f[(3 + a) * cn + k] = a < d ? vel[i * d + a] : 0.0;
            }
            // a wall particle's reference density is 1: its volume is the lattice one
            const double r0 = phase[i] == kWall ? 1.0 : s->prm.rho0[phase[i]];
            f[6 * cn + k] = mass ? mass[i] : r0 / s->sc.sigma0;
            f[7 * cn + k] = rho ? rho[i] : r0;
            f[8 * cn + k] = 0.0;
            ib[k] = (int32_t)i;
            ib[cn + k] = phase[i];
        }
        const int64_t o = s->p_off + i0;
        for (int q = 0; q < 9; ++q)
            HIPCHECK(hipMemcpyAsync(dst[q] + o, f + q * cn, sizeof(double) * m, hipMemcpyHostToDevice, P->stream));
        HIPCHECK(hipMemcpyAsync(P->A.id + o, ib, sizeof(int32_t) * m, hipMemcpyHostToDevice, P->stream));
        HIPCHECK(hipMemcpyAsync(P->A.phase + o, ib + cn, sizeof(int32_t) * m, hipMemcpyHostToDevice, P->stream));
        HIPCHECK(hipStreamSynchronize(P->stream));
    }
}

// Substeps of an advection step that starts from the per-fluid |v| maxima
// given: the advection step over the acoustic step of Eqs. 16-18, as the
// device takes them at the start of the step.  A scheduling estimate only:
// the device decides every step, and the acoustic step changes as the
// velocities do.
long long first_step_estimate(const SysConst& S, const double* vmax)
{
    double dt_ad = INFINITY, dt_ac = INFINITY;
    for (int f = 0; f < 2; ++f) {
        const double a = vmax[f] > 0.0 ? S.h / vmax[f] : INFINITY;
        dt_ad = std::min(dt_ad, std::min(S.cfl_ad * a, S.dtad_visc[f]));
        dt_ac = std::min(dt_ac, std::min(S.cfl_ac * (S.h / (S.c0 + vmax[f])), S.dtac_surf[f]));
    }
    if (!std::isfinite(dt_ad) || !(dt_ac > 0.0)) return 1;
    return (long long)std::min(1e6, std::max(1.0, std::ceil(dt_ad / dt_ac)));
}

void reset_dyn(rsph_system* s, bool keep_clock)
{
    rsph_pool* P = s->pool;
    HIPCHECK(hipStreamSynchronize(P->stream));
    SysDyn d{};
    if (keep_clock) HIPCHECK(hipMemcpy(&d, P->A.sd + s->row, sizeof(SysDyn), hipMemcpyDeviceToHost));
    d.health = 0;
    d.stepping = 0;
    d.binned = 0;
    d.displaced = 0;
    if (!keep_clock) d.n_displaced = 0;
    d.ksub_max = 0;
    d.state = kBoundary;
    d.sub_state = kIdle;
    d.ksub = 0;
    if (!keep_clock) {
        d.t = d.tau = d.dt_ad = d.dt_last = 0.0;
        d.n_sub = d.n_outer = 0;
        d.dt[0] = d.dt[1] = 0.0;
        d.vmax[0] = d.vmax[1] = 0.0;
    }
    d.target = d.n_outer;
    s->seen_outer = d.n_outer;
    s->seen_sub = d.n_sub;
    if (!keep_clock) s->sps = 0;
    s->first_sps = first_step_estimate(s->sc, s->v0max);
    HIPCHECK(hipMemcpy(P->A.sd + s->row, &d, sizeof(SysDyn), hipMemcpyHostToDevice));
}

// clears the evaluation's traces: stepping flags and the |v| accumulator
void clear_after_rebuild(rsph_system* s)
{
    rsph_pool* P = s->pool;
    HIPCHECK(hipStreamSynchronize(P->stream));
    SysDyn d;
    HIPCHECK(hipMemcpy(&d, P->A.sd + s->row, sizeof(SysDyn), hipMemcpyDeviceToHost));
    d.stepping = 0;
    d.health &= ~kHealthClose;
    HIPCHECK(hipMemcpy(P->A.sd + s->row, &d, sizeof(SysDyn), hipMemcpyHostToDevice));
}

// Rebuilds the neighbourhood of one system without changing its state and
// rejects inputs with particles closer than 1e-3 dp or overflowing lists.
void check_spacing(rsph_system* s)
{
    rsph_pool* P = s->pool;
    std::vector<int32_t> mask(P->systems.size(), 0);
    mask[s->row] = 1;
    set_mask(P, mask);
    rebuild(P, 1, -1);
    HIPCHECK(hipStreamSynchronize(P->stream));
    SysDyn d;
    HIPCHECK(hipMemcpy(&d, P->A.sd + s->row, sizeof(SysDyn), hipMemcpyDeviceToHost));
    const uint32_t bad = d.health;
    d.health = 0;
    d.stepping = 0;
    HIPCHECK(hipMemcpy(P->A.sd + s->row, &d, sizeof(SysDyn), hipMemcpyHostToDevice));
    if (bad & (kHealthClose | kHealthCoincident))
        fail(RSPH_EINVAL, "two particles are closer than 1e-3 dp");
    if (bad & kHealthNeighbours) fail(RSPH_EINVAL, "a particle has more neighbours than the list holds");
}

void make_pool(rsph_pool* P, int dim, int precision, size_t budget, void* stream)
{
    P->dim = dim;
    P->precision = precision;
    P->budget = budget;
    if (stream) {
        P->stream = (hipStream_t)stream;
        P->own_stream = false;
    } else {
        HIPCHECK(hipStreamCreate(&P->stream));
        P->own_stream = true;
    }
}

void destroy_pool(rsph_pool* P)
{
    if (!P) return;
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    for (auto& t : P->pending) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (auto e : P->event_pool) (void)hipEventDestroy(e);
    free_arrays(P);
    if (P->stage) (void)hipHostFree(P->stage);
    if (P->pin_dyn) (void)hipHostFree(P->pin_dyn);
    if (P->pin_targets) (void)hipHostFree(P->pin_targets);
    if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
    delete P;
}

// particle -> field readers
int field_width(int field, int d)
{
    switch (field) {
    case RSPH_FIELD_POS: case RSPH_FIELD_VEL: case RSPH_FIELD_ACC: case RSPH_FIELD_ACC_P:
    case RSPH_FIELD_ACC_S: case RSPH_FIELD_ACC_V: case RSPH_FIELD_GRADC: case RSPH_FIELD_DR:
        return d;
    case RSPH_FIELD_B:
        return d * d;
    default:
        return 1;
    }
}

template <typename T>
std::vector<T> dl(rsph_pool* P, const T* src, int64_t count)
{
    std::vector<T> v(count);
    HIPCHECK(hipStreamSynchronize(P->stream));
    if (count) HIPCHECK(hipMemcpy(v.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost));
    return v;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================

extern "C" {

void rsph_params_default(rsph_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->dim = 2;
    p->precision = RSPH_FP64;
    p->box[0] = p->box[1] = p->box[2] = 1.0;
    p->dp = 0.02;
    p->h_over_dp = 1.3;
    p->rho0[0] = p->rho0[1] = 1.0;
    p->eta[0] = p->eta[1] = 0.0;
    p->c0 = 1.0;
    p->gamma = 0.0;
    p->xi = -1.0;
    p->alpha_shift = 0.2;
    p->cfl_ad = 0.1;
    p->cfl_ac = 0.6;
}

const char* rsph_status_string(rsph_status s)
{
    switch (s) {
    case RSPH_OK: return "ok";
    case RSPH_EINVAL: return "invalid argument";
    case RSPH_ENOMEM: return "out of device memory";
    case RSPH_EDEVICE: return "device error";
    case RSPH_ESTATE: return "invalid state";
    case RSPH_ENUMERIC: return "numerical fault";
    case RSPH_EBUSY: return "busy: budget exhausted";
    }
    return "unknown status";
}

const char* rsph_last_error(const rsph_system* sys)
{
    return sys ? sys->err.c_str() : g_last_error.c_str();
}

rsph_status rsph_create_system(const rsph_params* params, void* hip_stream, rsph_system** out)
{
    return guarded(nullptr, [&] {
        if (!out) fail(RSPH_EINVAL, "out is NULL");
        *out = nullptr;
        validate_params(params);
        rsph_pool* P = new rsph_pool();
        try {
            make_pool(P, params->dim, params->precision, 0, hip_stream);
        } catch (...) {
            destroy_pool(P);
            throw;
        }
        P->standalone = true;
        rsph_system* s = new rsph_system();
        s->pool = P;
        s->owns_pool = true;
        s->prm = *params;
        s->sc = make_const(*params);
        s->ncells = s->sc.ncells;
        *out = s;
    });
}

rsph_status rsph_set_particles(rsph_system* s, int64_t n, const double* pos, const double* vel,
                               const int32_t* phase, const double* mass, const double* rho,
                               uint32_t opts)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (!s->owns_pool) fail(RSPH_ESTATE, "systems of a served pool take particles at admission");
        validate_particles(s->prm, n, pos, vel, phase, mass, rho);
        const SysConst sc_new = const_for_particles(s->prm, n, vel);
        rsph_pool* P = s->pool;
        const bool keep = (opts & RSPH_KEEP_CLOCK) && s->has_particles && s->row >= 0;
        s->has_particles = false;
        s->n = n;
        // standalone pool: size the arrays exactly for this system
        Layout L = plan({}, s);
        if (L.P != P->P_cap || L.C != P->C_cap) {
            std::vector<SysDyn> keepd;
            if (keep) keepd = read_dyn(P);
            free_arrays(P);
            alloc_arrays(P, L.P, L.C, 1);
            s->row = -1;
            repack(P, {s});
            if (keep) HIPCHECK(hipMemcpy(P->A.sd, keepd.data(), sizeof(SysDyn), hipMemcpyHostToDevice));
        } else {
            repack(P, {s});
        }
        s->has_particles = true;
        // the slot and cell placement of the packing stays; the constants
        // may change with c0 (a reset with new velocities under c0 = 0)
        const SysConst placed = s->sc;
        s->sc = sc_new;
        s->sc.p_off = placed.p_off;
        s->sc.c_off = placed.c_off;
        s->sc.fuse_dt = placed.fuse_dt;
        s->sc.p_n = n;
        set_fluid_masses(s, n, phase, mass);
        HIPCHECK(hipMemcpy((void*)(P->A.sc + s->row), &s->sc, sizeof(SysConst), hipMemcpyHostToDevice));
        upload_particles(s, pos, vel, phase, mass, rho);
        reset_dyn(s, keep);
        s->faulted = false;
        s->rates_valid = false;
        try {
            check_spacing(s);
        } catch (...) {
            s->has_particles = false;
            throw;
        }
    });
}

rsph_status rsph_set_drho(rsph_system* s, int64_t n, const double* drho)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (!s->has_particles) fail(RSPH_ESTATE, "no particles");
        if (n != s->n || !drho) fail(RSPH_EINVAL, "n must equal the particle count");
        rsph_pool* P = s->pool;
        std::vector<int32_t> id = dl(P, P->A.id + s->p_off, n);
        std::vector<double> v(n);
        for (int64_t k = 0; k < n; ++k) v[k] = drho[id[k]];
        HIPCHECK(hipMemcpy(P->A.drho + s->p_off, v.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    });
}

rsph_status rsph_step(rsph_system* s, int64_t n_outer)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (n_outer < 0) fail(RSPH_EINVAL, "n_outer must be >= 0");
        if (!s->has_particles) fail(RSPH_ESTATE, "no particles");
        if (s->faulted) fail(RSPH_ESTATE, "system is faulted; reset it with rsph_set_particles");
        if (n_outer == 0) return;
        rsph_pool* P = s->pool;
        s->rates_valid = false;
        std::vector<SysDyn> d = read_dyn(P);
        std::vector<long long> targets(P->systems.size(), -1);
        targets[s->row] = d[s->row].n_outer + n_outer;
        set_targets(P, targets);
        std::vector<long long> left(P->systems.size(), 0);
        left[s->row] = n_outer;
        const uint32_t h = run_to_targets(P, left);
        if (h & kFaultBits) {
            s->faulted = true;
            char buf[128];
            std::snprintf(buf, sizeof buf, "health check tripped (bits 0x%x)", h);
            fail(RSPH_ENUMERIC, buf);
        }
    });
}

rsph_status rsph_eval_rates(rsph_system* s)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (!s->has_particles) fail(RSPH_ESTATE, "no particles");
        rsph_pool* P = s->pool;
        const Launch L = launch_of(P);
        std::vector<int32_t> mask(P->systems.size(), 0);
        mask[s->row] = 1;
        set_mask(P, mask);
        rebuild(P, 1, -1);
        DevArrays A = kernel_view(P);
        A.work = nullptr;
        A.mode = 1;
        launch_advection(L, A, Ev{});
        launch_shift(L, A, Ev{});
        launch_colour(L, A, Ev{});
        launch_force(L, A, Ev{});
        launch_continuity(L, A, Ev{}, -1);
        clear_after_rebuild(s);
        s->rates_valid = true;
    });
}

rsph_status rsph_read_observables(rsph_system* s, rsph_observables* out)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (!out) fail(RSPH_EINVAL, "out is NULL");
        if (!s->has_particles) fail(RSPH_ESTATE, "no particles");
        rsph_pool* P = s->pool;
        const Launch L = launch_of(P);
        launch_observables(L, P->A);
        double o[kObsOut];
        SysDyn d;
        HIPCHECK(hipStreamSynchronize(P->stream));
        HIPCHECK(hipMemcpy(o, P->A.obs_out + (int64_t)s->row * kObsOut, sizeof o, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(&d, P->A.sd + s->row, sizeof d, hipMemcpyDeviceToHost));
        std::memset(out, 0, sizeof(*out));
        out->t = d.t;
        out->n_outer = d.n_outer;
        out->n_sub = d.n_sub;
        out->dt_ad = d.dt_ad;
        out->dt_ac = d.dt_last;
        for (int a = 0; a < 3; ++a) out->momentum[a] = o[a];
        out->kinetic = o[3];
        out->mass[0] = o[4];
        out->mass[1] = o[5];
        out->volume[0] = o[6];
        out->volume[1] = o[7];
        out->vmax[0] = o[8];
        out->vmax[1] = o[9];
        for (int a = 0; a < 3; ++a) out->centroid[a] = o[10 + a];
        out->r_eq = o[13];
        const double m2[6] = {o[16], o[17], o[18], o[19], o[20], o[21]};
        const int idx[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
        for (int q = 0; q < 9; ++q) out->moment2[q] = m2[idx[q]];
        out->n_in = o[23];
        out->n_out = o[25];
        out->p_in = o[23] > 0 ? o[22] / o[23] : 0.0;
        out->p_out = o[25] > 0 ? o[24] / o[25] : 0.0;
        out->health = d.health;
        out->displaced_steps = (uint32_t)std::min<long long>(d.n_displaced, UINT32_MAX);
    });
}

rsph_status rsph_read_particles(rsph_system* s, int32_t field, int64_t n, double* out)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (!out) fail(RSPH_EINVAL, "out is NULL");
        if (!s->has_particles) fail(RSPH_ESTATE, "no particles");
        if (n != s->n) fail(RSPH_EINVAL, "n must equal the particle count");
        if (field < 0 || field >= RSPH_FIELD_COUNT) fail(RSPH_EINVAL, "unknown field");
        if (field >= RSPH_FIELD_ACC && field <= RSPH_FIELD_SIGMA && !s->rates_valid)
            fail(RSPH_ESTATE, "rates are read after rsph_eval_rates");
        rsph_pool* P = s->pool;
        HIPCHECK(hipStreamSynchronize(P->stream));
        const DevArrays& A = P->A;
        const int d = s->prm.dim;
        const int w = field_width(field, d);
        const int64_t o = s->p_off;
        std::vector<int32_t> id = dl(P, A.id + o, n);
        std::vector<double> tmp((size_t)n * w);
        auto soa = [&](double* const* arr) {
            for (int a = 0; a < d; ++a) {
                std::vector<double> v = dl(P, arr[a] + o, n);
                for (int64_t k = 0; k < n; ++k) tmp[(size_t)k * w + a] = v[k];
            }
        };
        auto aos3 = [&](const double* arr) {
            std::vector<double> v = dl(P, arr + 3 * o, 3 * n);
            for (int64_t k = 0; k < n; ++k)
                for (int a = 0; a < d; ++a) tmp[(size_t)k * w + a] = v[3 * k + a];
        };
        auto one = [&](const double* arr) {
            std::vector<double> v = dl(P, arr + o, n);
            for (int64_t k = 0; k < n; ++k) tmp[k] = v[k];
        };
        switch (field) {
        case RSPH_FIELD_POS: soa(A.pos); break;
        case RSPH_FIELD_VEL: soa(A.vel); break;
        case RSPH_FIELD_RHO: one(A.rho); break;
        case RSPH_FIELD_DRHO: one(A.drho); break;
        case RSPH_FIELD_MASS: one(A.mass); break;
        case RSPH_FIELD_P: {
            std::vector<double> r = dl(P, A.rho + o, n);
            std::vector<int32_t> ph = dl(P, A.phase + o, n);
            for (int64_t k = 0; k < n; ++k)
                tmp[k] = ph[k] == kWall ? 0.0 : s->sc.c0sq * (r[k] - s->sc.rho0[ph[k]]);
            break;
        }
        case RSPH_FIELD_PHASE: {
            std::vector<int32_t> ph = dl(P, A.phase + o, n);
            for (int64_t k = 0; k < n; ++k) tmp[k] = (double)ph[k];
            break;
        }
        case RSPH_FIELD_ACC: aos3(A.r_acc); break;
        case RSPH_FIELD_ACC_P: aos3(A.r_accp); break;
        case RSPH_FIELD_ACC_S: aos3(A.r_accs); break;
        case RSPH_FIELD_ACC_V: aos3(A.r_accv); break;
        case RSPH_FIELD_GRADC: aos3(A.r_gradc); break;
        case RSPH_FIELD_DR: aos3(A.r_dr); break;
        case RSPH_FIELD_RATE_DRHO: one(A.r_drho); break;
        case RSPH_FIELD_SIGMA: one(A.r_sigma); break;
        case RSPH_FIELD_B: {
            std::vector<double> v = dl(P, A.r_b + 9 * o, 9 * n);
            for (int64_t k = 0; k < n; ++k)
                for (int q = 0; q < w; ++q) tmp[(size_t)k * w + q] = v[9 * k + q];
            break;
        }
        case RSPH_FIELD_NNB: {
            std::vector<int32_t> c = dl(P, A.ncount + o, n);
            for (int64_t k = 0; k < n; ++k) tmp[k] = (double)c[k];
            break;
        }
        case RSPH_FIELD_FLAGS: {
            std::vector<uint8_t> c = dl(P, A.flags + o, n);
            for (int64_t k = 0; k < n; ++k) tmp[k] = (double)c[k];
            break;
        }
        }
        for (int64_t k = 0; k < n; ++k)
            for (int q = 0; q < w; ++q) out[(size_t)id[k] * w + q] = tmp[(size_t)k * w + q];
    });
}

rsph_status rsph_read_binning(rsph_system* s, int64_t n, uint32_t* key, int64_t* rank)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (!key || !rank) fail(RSPH_EINVAL, "NULL output");
        if (!s->has_particles) fail(RSPH_ESTATE, "no particles");
        if (n != s->n) fail(RSPH_EINVAL, "n must equal the particle count");
        rsph_pool* P = s->pool;
        HIPCHECK(hipStreamSynchronize(P->stream));
        const int64_t o = s->p_off;
        std::vector<int32_t> id = dl(P, P->A.id + o, n);
        std::vector<int32_t> perm = dl(P, P->A.perm + o, n);
        std::vector<uint32_t> k_old = dl(P, P->A.key, P->A.P);
        for (int64_t k = 0; k < n; ++k) {
            key[id[k]] = k_old[perm[k]];
            rank[id[k]] = k;
        }
    });
}

rsph_status rsph_read_neighbours(rsph_system* s, int64_t n, int64_t cap, int64_t* start, int64_t* idx)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (!start || !idx) fail(RSPH_EINVAL, "NULL output");
        if (!s->has_particles) fail(RSPH_ESTATE, "no particles");
        if (n != s->n) fail(RSPH_EINVAL, "n must equal the particle count");
        rsph_pool* P = s->pool;
        HIPCHECK(hipStreamSynchronize(P->stream));
        const DevArrays& A = P->A;
        const int64_t o = s->p_off;
        std::vector<int32_t> id = dl(P, A.id, A.P);
        std::vector<int32_t> cnt = dl(P, A.ncount + o, n);
        const int64_t w0 = o / kWave, w1 = (o + n + kWave - 1) / kWave;
        std::vector<uint32_t> nb = dl(P, A.nbr + w0 * A.kmax * kWave, (w1 - w0) * A.kmax * kWave);
        std::vector<int64_t> count(n);
        for (int64_t k = 0; k < n; ++k) count[id[o + k]] = cnt[k];
        start[0] = 0;
        for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + count[i];
        if (start[n] > cap) fail(RSPH_EINVAL, "cap is too small");
        for (int64_t k = 0; k < n; ++k) {
            const int64_t slot = o + k;
            const int64_t w = slot / kWave - w0, lane = slot % kWave;
            const int64_t dst = start[id[slot]];
            for (int q = 0; q < cnt[k]; ++q)
                idx[dst + q] = id[nb[(w * A.kmax + q) * kWave + lane] & kNbrIndexMask];
        }
    });
}

rsph_status rsph_set_launch_mode(rsph_system* s, int32_t mode)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (mode != RSPH_LAUNCH_GRAPH && mode != RSPH_LAUNCH_EAGER) fail(RSPH_EINVAL, "unknown launch mode");
        rsph_pool* P = s->pool;
        HIPCHECK(hipStreamSynchronize(P->stream));
        P->graphs = mode == RSPH_LAUNCH_GRAPH;
        if (!P->graphs) drop_graphs(P);
    });
}

rsph_status rsph_set_kernel_timing(rsph_system* s, int32_t enable)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        rsph_pool* P = s->pool;
        collect_timing(P);
        P->timing = enable != 0;
        P->timing_mask = (uint32_t)enable | (1u << RSPH_KERNEL_EVENT_FLOOR);
        for (int k = 0; k < RSPH_KERNEL_COUNT; ++k) {
            P->t_launches[k] = 0;
            P->t_ms[k] = 0.0;
        }
        if (P->timing) {
            // the fixed cost of a dispatch bracketed by timing events
            for (int q = 0; q < 32; ++q) {
                TimeScope t(P, RSPH_KERNEL_EVENT_FLOOR, -1);
                launch_empty(launch_of(P), t.ev);
            }
            collect_timing(P);
        }
    });
}

rsph_status rsph_read_kernel_timing(rsph_system* s, int64_t* launches, double* ms)
{
    if (!s) return RSPH_EINVAL;
    return guarded(&s->err, [&] {
        if (!launches || !ms) fail(RSPH_EINVAL, "NULL output");
        rsph_pool* P = s->pool;
        collect_timing(P);
        for (int k = 0; k < RSPH_KERNEL_COUNT; ++k) {
            launches[k] = P->t_launches[k];
            ms[k] = P->t_ms[k];
        }
    });
}

void rsph_destroy_system(rsph_system* s)
{
    if (!s) return;
    if (s->owns_pool) {
        destroy_pool(s->pool);
        delete s;
        return;
    }
    (void)rsph_pool_release(s->pool, s);
}

// ---- serving ----------------------------------------------------------------

rsph_status rsph_pool_create(int32_t dim, int32_t precision, size_t budget, void* hip_stream, rsph_pool** out)
{
    return guarded(nullptr, [&] {
        if (!out) fail(RSPH_EINVAL, "out is NULL");
        *out = nullptr;
        if (dim != 2 && dim != 3) fail(RSPH_EINVAL, "dim must be 2 or 3");
        if (precision != RSPH_FP64 && precision != RSPH_MIXED) fail(RSPH_EINVAL, "bad precision");
        rsph_pool* P = new rsph_pool();
        try {
            make_pool(P, dim, precision, budget, hip_stream);
        } catch (...) {
            destroy_pool(P);
            throw;
        }
        *out = P;
    });
}

rsph_status rsph_pool_admit(rsph_pool* P, const rsph_params* params, int64_t n, const double* pos,
                            const double* vel, const int32_t* phase, const double* mass, rsph_system** out)
{
    if (!P) return RSPH_EINVAL;
    return guarded(&P->err, [&] {
        if (!out) fail(RSPH_EINVAL, "out is NULL");
        *out = nullptr;
        validate_params(params);
        if (params->dim != P->dim || params->precision != P->precision)
            fail(RSPH_EINVAL, "system dim and precision must match the pool's");
        validate_particles(*params, n, pos, vel, phase, mass, nullptr);
        const SysConst sc = const_for_particles(*params, n, vel);
        rsph_system* s = new rsph_system();
        s->pool = P;
        s->prm = *params;
        s->sc = sc;
        s->ncells = s->sc.ncells;
        s->n = n;
        std::vector<rsph_system*> members = P->systems;
        members.push_back(s);
        try {
            repack(P, members);
            s->has_particles = true;
            s->sc.p_n = n;
            set_fluid_masses(s, n, phase, mass);
            HIPCHECK(hipMemcpy((void*)(P->A.sc + s->row), &s->sc, sizeof(SysConst), hipMemcpyHostToDevice));
            upload_particles(s, pos, vel, phase, mass, nullptr);
            reset_dyn(s, false);
            check_spacing(s);
        } catch (...) {
            std::vector<rsph_system*> back(P->systems.begin(), P->systems.end());
            back.erase(std::remove(back.begin(), back.end(), s), back.end());
            if (s->row >= 0) {
                try {
                    repack(P, back);
                } catch (...) {
                }
            }
            delete s;
            throw;
        }
        *out = s;
    });
}

rsph_status rsph_pool_step(rsph_pool* P, rsph_system* const* systems, const int64_t* n_outer, int32_t count)
{
    if (!P) return RSPH_EINVAL;
    return guarded(&P->err, [&] {
        if (count < 0 || (count > 0 && (!systems || !n_outer))) fail(RSPH_EINVAL, "bad arguments");
        // advection steps done, as the host last read them: every stepping
        // call ends with a read, and a reset sets them
        std::vector<long long> done(P->systems.size());
        for (size_t r = 0; r < done.size(); ++r) done[r] = P->systems[r]->seen_outer;
        std::vector<long long> targets(P->systems.size(), -1);
        int64_t most = 0;
        for (int k = 0; k < count; ++k) {
            rsph_system* s = systems[k];
            if (!s || s->pool != P || s->row < 0) fail(RSPH_EINVAL, "system is not in this pool");
            if (s->faulted) fail(RSPH_ESTATE, "a system of the batch is faulted");
            if (n_outer[k] < 0) fail(RSPH_EINVAL, "n_outer must be >= 0");
            const long long base = targets[s->row] >= 0 ? targets[s->row] : done[s->row];
            targets[s->row] = base + n_outer[k];
            most = std::max<int64_t>(most, targets[s->row] - done[s->row]);
            s->rates_valid = false;
        }
        if (most == 0) return;
        set_targets(P, targets);
        std::vector<long long> left(P->systems.size(), 0);
        for (size_t r = 0; r < left.size(); ++r)
            if (targets[r] >= 0) left[r] = targets[r] - done[r];
        const uint32_t h = run_to_targets(P, left);
        if (h & kFaultBits) {
            std::vector<SysDyn> dd = read_dyn(P);
            std::string names;
            for (size_t r = 0; r < dd.size(); ++r)
                if (dd[r].health & kFaultBits) {
                    P->systems[r]->faulted = true;
                    names += " " + std::to_string(r);
                }
            P->err = "health check tripped in pool rows" + names;
            for (int k = 0; k < count; ++k)
                if (systems[k]->faulted) fail(RSPH_ENUMERIC, P->err);
        }
    });
}

size_t rsph_pool_bytes(const rsph_pool* P) { return P ? P->bytes : 0; }

rsph_status rsph_step_counts(const rsph_system* s, int64_t* n_outer, int64_t* n_sub, int64_t* substeps_per_step)
{
    if (!s || !n_outer || !n_sub || !substeps_per_step) return RSPH_EINVAL;
    *n_outer = s->seen_outer;
    *n_sub = s->seen_sub;
    *substeps_per_step = s->sps > 0 ? s->sps : (s->seen_outer == 0 ? s->first_sps : 0);
    return RSPH_OK;
}

rsph_status rsph_pool_release(rsph_pool* P, rsph_system* s)
{
    if (!P || !s) return RSPH_EINVAL;
    return guarded(&P->err, [&] {
        if (s->pool != P || s->owns_pool) fail(RSPH_EINVAL, "system is not in this pool");
        std::vector<rsph_system*> members;
        for (auto* m : P->systems)
            if (m != s) members.push_back(m);
        repack(P, members);
        delete s;
    });
}

void rsph_pool_destroy(rsph_pool* P)
{
    if (!P) return;
    for (auto* s : P->systems) delete s;
    P->systems.clear();
    destroy_pool(P);
}

}  // extern "C"

// ---- evaluation without allocation ------------------------------------------

namespace {

// The working memory of rsph_eval_rates_noalloc: one fixed array per device,
// held until the process ends.  Host code must not pass its name to a kernel
// (that is a host-side stand-in); the device address comes from
// hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_lock;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_address()
{
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(RSPH_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> g(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) fail(RSPH_EDEVICE, "scratch array has no device address");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// Carves the arrays of plan_arrays out of the scratch array, 256-byte aligned.
struct ScratchCarver {
    char* base;
    size_t cap;
    size_t bytes = 0;
    template <typename T>
    T* take(size_t count)
    {
        const size_t b = (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
        if (bytes + b > cap) fail(RSPH_EINVAL, "input too large for the evaluation scratch");
        T* p = (T*)(base + bytes);
        bytes += b;
        return p;
    }
};

// Bytes the carver needs for one system of n particles (arrays 256-byte aligned)
struct CountCarver {
    size_t bytes = 0;
    template <typename T>
    T* take(size_t count)
    {
        bytes += (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
        return nullptr;
    }
};

}  // namespace

extern "C" rsph_status rsph_eval_rates_noalloc(const rsph_params* params, int64_t n, const double* pos,
                                               const double* vel, const int32_t* phase, const double* mass,
                                               const double* rho, double* acc, double* drho_rate,
                                               void* hip_stream)
{
    return guarded(nullptr, [&] {
        validate_params(params);
        if (!(params->c0 > 0)) fail(RSPH_EINVAL, "this entry point needs c0 > 0");
        if (n < 1) fail(RSPH_EINVAL, "n must be >= 1");
        if (n > kMaxSlots) fail(RSPH_EINVAL, "too many particles (2^26 per pool)");
        if (!pos || !vel || !phase || !acc || !drho_rate) fail(RSPH_EINVAL, "pos, vel, phase, acc and drho are required");
        char* base = (char*)scratch_address();
        // a pool of one system whose arrays live in the scratch array
        rsph_pool P;
        P.dim = params->dim;
        P.precision = params->precision;
        P.stream = (hipStream_t)hip_stream;
        P.standalone = true;
        P.graphs = false;
        rsph_system s;
        s.pool = &P;
        s.prm = *params;
        s.sc = make_const(*params);
        s.ncells = s.sc.ncells;
        s.n = n;
        Layout L = plan({}, &s);
        CountCarver count;
        DevArrays probe;
        int32_t *m0 = nullptr, *w0 = nullptr;
        long long* t0 = nullptr;
        const size_t need = plan_arrays(count, P.dim, P.precision, probe, m0, t0, w0, L.P, L.C, 1) + 256;
        if (need > kScratchBytes) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "%lld particles need %zu bytes of evaluation scratch; it holds %zu",
                          (long long)n, need, kScratchBytes);
            fail(RSPH_EINVAL, buf);
        }
        ScratchCarver carve{base, kScratchBytes};
        plan_arrays(carve, P.dim, P.precision, P.A, P.d_mask, P.d_targets, P.work_dev, L.P, L.C, 1);
        // what the load finds: invalid input, walls, per-fluid mass range
        unsigned long long* probe_d = carve.take<unsigned long long>(kLoadProbeWords);
        P.P_cap = L.P;
        P.C_cap = L.C;
        P.S_cap = 1;
        const Launch Lc = launch_of(&P);
        // the scratch keeps the last call's contents: clear what starts at zero
        launch_fill_i32(Lc, P.A.cell_cnt, L.C, 0);
        launch_fill_i32(Lc, P.work_dev, P.A.work_cap, 0);
        launch_fill_i32(Lc, (int32_t*)probe_d, 2, 0);
        launch_fill_i32(Lc, (int32_t*)(probe_d + 1), 4, -1);
        launch_fill_i32(Lc, (int32_t*)(probe_d + 3), 4, 0);
        repack(&P, {&s});
        s.has_particles = true;
        s.sc.p_n = n;
        HIPCHECK(hipMemcpyAsync((void*)(P.A.sc + s.row), &s.sc, sizeof(SysConst), hipMemcpyHostToDevice, P.stream));
        launch_load_particles(Lc, P.A, s.p_off, n, pos, vel, phase, mass, rho, s.sc.box, s.sc.rho0, s.sc.sigma0,
                              probe_d);
        unsigned long long probe_h[kLoadProbeWords] = {};
        HIPCHECK(hipMemcpyAsync(probe_h, probe_d, sizeof probe_h, hipMemcpyDeviceToHost, P.stream));
        HIPCHECK(hipStreamSynchronize(P.stream));
        if (probe_h[0] & 1ull)
            fail(RSPH_EINVAL, "a phase outside {0,1,2}, a non-finite value, or a mass or density <= 0");
        // the same choice of pair passes as the allocating path makes on the host
        s.has_walls = (probe_h[0] & 2ull) != 0;
        s.uniform_mass = true;
        for (int f = 0; f < 2; ++f) {
            if (probe_h[1 + f] > probe_h[3 + f]) continue;  // no particle of this fluid
            if (probe_h[1 + f] != probe_h[3 + f]) s.uniform_mass = false;
            else std::memcpy(&s.sc.mphase[f], &probe_h[1 + f], sizeof(double));
        }
        HIPCHECK(hipMemcpyAsync((void*)(P.A.sc + s.row), &s.sc, sizeof(SysConst), hipMemcpyHostToDevice, P.stream));
        reset_dyn(&s, false);
        check_spacing(&s);
        // one evaluation, as rsph_eval_rates
        std::vector<int32_t> mask(1, 1);
        set_mask(&P, mask);
        rebuild(&P, 1, -1);
        DevArrays A = kernel_view(&P);
        A.work = nullptr;
        A.mode = 1;
        launch_advection(Lc, A, Ev{});
        launch_shift(Lc, A, Ev{});
        launch_colour(Lc, A, Ev{});
        launch_force(Lc, A, Ev{});
        launch_continuity(Lc, A, Ev{}, -1);
        launch_store_rates(Lc, A, s.p_off, n, acc, drho_rate);
        HIPCHECK(hipStreamSynchronize(P.stream));
        P.systems.clear();
    });
}
