// rsph_kernels.hip -- HIP kernels for gfx950 (CDNA4) of the Riemann-SPH
// multiphase surface-tension method (arXiv 2503.16082).
//
// Pair passes use G = 4 lanes per particle slot, wave64,
// 256-thread blocks.  Blocks are remapped
// so that each of the 8 XCDs works on one contiguous eighth of the slot range:
// particles are cell-sorted, so neighbour gathers of a block mostly hit the L2
// of its own XCD.  Pair loops gather-only: every particle sums its own
// neighbours in a fixed order, so results are deterministic and no floating
// point atomics are used (the only atomics are integer ones: the counting
// sort's cell counters, whose arrival order the rank pass makes canonical,
// health and work flags, and the LDS cell bounds of the neighbour staging).
//
// Precision forms: R = double (FP64 form) or R = float (mixed form: FP32 pair
// arithmetic on split positions, FP64 state updates).  D = 2 or 3.
#include <math.h>

#include <hip/hip_ext.h>

#include <utility>

#include "rsph_internal.h"

namespace rsph {

template <typename R>
struct alignas(4 * sizeof(R)) Q4 {
    R x, y, z, w;
};

// ---------------------------------------------------------------------------
// indexing helpers
// ---------------------------------------------------------------------------

// Consecutive logical blocks on the same XCD (workgroups are dispatched
// round-robin over the 8 XCDs); gridDim.x is a multiple of 8.
__device__ __forceinline__ int64_t logical_block()
{
    const int64_t per = gridDim.x >> 3;
    const int64_t b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

// system of the 64-slot block w (-1: none): from the per-wave table, or
// without a load when the pool holds a single system
__device__ __forceinline__ int system_of_wave(const DevArrays& A, int64_t w)
{
    if (A.one_sys_waves > 0) return w < A.one_sys_waves ? 0 : -1;
    return A.wave_sys[w];
}

struct Slot {
    int64_t i;   // slot index
    int s;       // system (wave-uniform), -1 if none
    bool lane;   // slot holds a particle
};

__device__ __forceinline__ Slot slot_of(const DevArrays& A)
{
    Slot c;
    c.i = logical_block() * kBlock + threadIdx.x;
    c.s = -1;
    c.lane = false;
    if (c.i >= A.P) return c;
    int s = system_of_wave(A, c.i >> 6);
    s = __builtin_amdgcn_readfirstlane(s);
    c.s = s;
    if (s < 0) return c;
    const SysConst& S = A.sc[s];
    c.lane = c.i < S.p_off + S.p_n;
    return c;
}

// Iterates lane g of particle i's group over list entries g, g + G, ... in
// order.  Entries are taken CH at a time: the CH indices are loaded together,
// then the neighbour records of all CH (load(slot)), then body(entry, record)
// runs for each valid entry in list order.  The gathers of CH iterations are thus
// in flight at once, while every sum accumulates in the order of the list.
// Entries past the count reuse the group's first entry (a valid slot), so every
// load stays inside the arrays.
template <int G, int CH, typename Load, typename Body>
__device__ __forceinline__ void for_neighbours(const DevArrays& A, int64_t i, int g, int cnt,
                                               Load&& load, Body&& body)
{
    const uint32_t* list = A.nbr + ((i >> 6) * A.kmax) * kWave + (i & 63);
    for (int k0 = g; k0 < cnt; k0 += G * CH) {
        uint32_t jb[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int k = k0 + u * G;
            jb[u] = list[(int64_t)(k < cnt ? k : k0) * kWave];
        }
        decltype(load(0u)) rec[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) rec[u] = load(jb[u] & kNbrIndexMask);
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (k0 + u * G < cnt) body(jb[u], rec[u]);
    }
}

template <typename R, int N>
struct Recs {
    Q4<R> q[N];
};

// The FP64 position of a slot as the rank pass leaves it, with the phase's
// two bits in the sign bits of x and y (positions are wrapped into [0, L), so
// their signs are free): 16 bytes per slot in 2D; in 3D a 32-byte slot of
// which a reader takes the 24 bytes of x, y, z (two loads, one cache line).
template <int D>
__device__ __forceinline__ void store_pos(const DevArrays& A, int64_t j, const double* x, int ph)
{
    const double x0 = (ph & 1) ? -x[0] : x[0];
    const double x1 = (ph & 2) ? -x[1] : x[1];
    if constexpr (D == 2) ((double2*)A.xd)[j] = double2{x0, x1};
    else ((double4*)A.xd)[j] = double4{x0, x1, x[2], 0.0};
}

// The fixed-point offset of slot j from its cell corner along each axis, in
// units of cell / 2^31 (31 bits, within 5e-10 of a cell of the FP64 value),
// with phase bit 0 and 1 in bit 31 of the x and y words: 12 bytes that give a
// pair distance to FP64 precision of about 1e-9 h, the mixed form's input to
// the 3D density summation.
struct U3 {
    uint32_t x, y, z;
};

__device__ __forceinline__ int cell_of(double x, const SysConst& S, int a);

__device__ __forceinline__ void store_xq(const DevArrays& A, int64_t j, const double* x, int ph, const SysConst& S)
{
    uint32_t u[3];
    for (int a = 0; a < 3; ++a) {
        const double t = (x[a] - (double)cell_of(x[a], S, a) * S.cell[a]) * (2147483648.0 * S.inv_cell[a]);
        u[a] = (uint32_t)fmin(fmax(rint(t), 0.0), 2147483647.0);
    }
    ((U3*)A.xq)[j] = U3{u[0] | ((uint32_t)(ph & 1) << 31), u[1] | ((uint32_t)(ph & 2) << 30), u[2]};
}

// FP64 position of slot j from its packed record, and its phase
template <int D>
__device__ __forceinline__ void load_pos(const DevArrays& A, int64_t j, double* x, int* ph = nullptr)
{
    double2 q;
    if constexpr (D == 2) {
        q = ((const double2*)A.xd)[j];
        x[2] = 0.0;
    } else {
        q = ((const double2*)A.xd)[2 * j];
        x[2] = A.xd[4 * j + 2];
    }
    x[0] = fabs(q.x);
    x[1] = fabs(q.y);
    if (ph) *ph = (signbit(q.x) ? 1 : 0) | (signbit(q.y) ? 2 : 0);
}

struct Pos3 {
    double x[3];
    int ph;
};

// ---------------------------------------------------------------------------
// kernel function (Wendland C2): W = alpha (1 - q/2)^4 (1 + 2q), q = r/h < 2
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R wendland_dw(R q, R coef)
{
    R a = R(1) - R(0.5) * q;
    return coef * q * a * a * a;  // coef = -5 alpha / h
}

__device__ __forceinline__ double wendland_w(double q, double alpha)
{
    double a = 1.0 - 0.5 * q;
    return alpha * a * a * a * a * (1.0 + 2.0 * q);
}

// ---------------------------------------------------------------------------
// frozen geometry records (phase 0, 1: the fluids; 2: a wall particle)
//   FP64: {x, y, z, phase + 4 * interface}
//   mixed: the offsets from the cell corner, |x - cx*cell|, |y - cy*cell|,
//          |z - cz*cell| (z: 0 in 2D), whose sign bits, free since an offset
//          is never negative, carry phase bit 0, phase bit 1 and the
//          interface bit; 12 bytes in 3D, a 16-byte record in 2D
// ---------------------------------------------------------------------------

struct F3 {
    float x, y, z;
};

template <typename R, int D>
struct GeoT {
    using T = Q4<R>;
};
template <>
struct GeoT<float, 3> {
    using T = F3;
};

// one neighbour's frozen-geometry record and N further 16-byte records
template <typename GT, typename R, int N>
struct GRecs {
    GT g;
    Q4<R> q[N];
};

template <typename R>
struct Geo;

template <>
struct Geo<double> {
    // w = phase + 4 * (particle has a neighbour of the other fluid)
    template <int D>
    __device__ static void store(void* geo, int64_t i, const double* x, int ph, bool iface, const SysConst& S,
                                 const int* c)
    {
        (void)S;
        (void)c;
        ((Q4<double>*)geo)[i] = Q4<double>{x[0], x[1], x[2], (double)(ph + (iface ? 4 : 0))};
    }
    __device__ static int phase(const Q4<double>& g) { return (int)g.w & 3; }
    __device__ static bool interface(const Q4<double>& g) { return ((int)g.w >> 2) != 0; }
    template <int D, typename GI, typename GJ>
    __device__ static void rij(const GI& gi, const GJ& gj, uint32_t e, const SysConst& S, const double* cellr,
                               double* r)
    {
        (void)e;
        (void)cellr;
        double d = gi.x - gj.x;
        if (d > S.half_box[0]) d -= S.box[0];
        else if (d < -S.half_box[0]) d += S.box[0];
        r[0] = d;
        d = gi.y - gj.y;
        if (d > S.half_box[1]) d -= S.box[1];
        else if (d < -S.half_box[1]) d += S.box[1];
        r[1] = d;
        if (D == 3) {
            d = gi.z - gj.z;
            if (d > S.half_box[2]) d -= S.box[2];
            else if (d < -S.half_box[2]) d += S.box[2];
            r[2] = d;
        } else {
            r[2] = 0.0;
        }
    }
};

template <>
struct Geo<float> {
    template <int D>
    __device__ static void store(void* geo, int64_t i, const double* x, int ph, bool iface, const SysConst& S,
                                 const int* c)
    {
        float o[3];
        // an offset is x - c cell >= 0 up to the rounding of the cell index
        // (below one ulp of x): its magnitude is kept, its sign bit set free
        for (int a = 0; a < 3; ++a) o[a] = fabsf((float)(x[a] - (double)c[a] * S.cell[a]));
        const bool bit[3] = {(ph & 1) != 0, (ph & 2) != 0, iface};
        for (int a = 0; a < 3; ++a) o[a] = bit[a] ? -o[a] : o[a];
        if constexpr (D == 3) ((F3*)geo)[i] = F3{o[0], o[1], o[2]};
        else ((Q4<float>*)geo)[i] = Q4<float>{o[0], o[1], o[2], 0.f};
    }
    template <typename GT>
    __device__ static int phase(const GT& g)
    {
        return (int)((__float_as_uint(g.x) >> 31) | ((__float_as_uint(g.y) >> 30) & 2u));
    }
    template <typename GT>
    __device__ static bool interface(const GT& g)
    {
        return (__float_as_uint(g.z) >> 31) != 0;
    }
    // r_ij = (o_i - o_j) + (c_i - c_j) cell, the cell differences (periodic
    // wrap included) taken from the list entry e
    template <int D, typename GI, typename GJ>
    __device__ static void rij(const GI& gi, const GJ& gj, uint32_t e, const SysConst& S, const float* cellr,
                               float* r)
    {
        (void)S;
        // each 2-bit field holds 1 - dx (dx the stencil offset, -1..1); with
        // its low bit flipped it is dx in two's complement, which a signed
        // bit-field extract returns: r = (o_i - o_j) - dx cell, the same
        // single rounding as (o_i - o_j) + (1 - dx - 1) cell
        const uint32_t f = e ^ 0x54000000u;
        r[0] = (fabsf(gi.x) - fabsf(gj.x)) - (float)((int32_t)(f << 4) >> 30) * cellr[0];
        r[1] = (fabsf(gi.y) - fabsf(gj.y)) - (float)((int32_t)(f << 2) >> 30) * cellr[1];
        if (D == 3) r[2] = (fabsf(gi.z) - fabsf(gj.z)) - (float)((int32_t)f >> 30) * cellr[2];
        else r[2] = 0.0f;
    }
};

template <typename R>
__device__ __forceinline__ R rsqrt_r(R x);
template <>
__device__ __forceinline__ double rsqrt_r<double>(double x) { return rsqrt(x); }
template <>
__device__ __forceinline__ float rsqrt_r<float>(float x) { return rsqrtf(x); }

// 1/r for a squared pair distance: in FP32 the hardware reciprocal square root
// alone (within 1 ulp), without the scaling rsqrtf adds for denormal
// arguments, which a pair distance never is (pairs closer than 1e-9 h are
// flagged).  Squared gradient norms can be denormal and take rsqrt_r.
template <typename R>
__device__ __forceinline__ R rsqrt_dist(R r2);
template <>
__device__ __forceinline__ double rsqrt_dist<double>(double r2) { return rsqrt(r2); }
template <>
__device__ __forceinline__ float rsqrt_dist<float>(float r2) { return __builtin_amdgcn_rsqf(r2); }

// 1/x: in FP32 the hardware reciprocal (within 1 ulp; the arguments here are
// densities and sums of them, never denormal), in FP64 the exact quotient
template <typename R>
__device__ __forceinline__ R recip(R x);
template <>
__device__ __forceinline__ double recip<double>(double x) { return 1.0 / x; }
template <>
__device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int cell_of(double x, const SysConst& S, int a)
{
    int64_t k = (int64_t)floor(__dmul_rn(x, S.inv_cell[a]));
    if (k < 0) k = 0;
    if (k > S.ncell[a] - 1) k = S.ncell[a] - 1;
    return (int)k;
}

// wave-wide max of non-negative doubles through their bit patterns
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

__device__ __forceinline__ void flag_health(SysDyn& D, uint32_t bits)
{
    atomicOr(&D.health, bits);
}

// lanes per particle in the pair passes: a particle's neighbour list is split
// over G consecutive lanes, whose partial sums are combined by a butterfly of
// xor-shuffles (fixed order, identical in every lane of the group)
#ifndef RSPH_LANES_2D
#define RSPH_LANES_2D 4
#endif
#ifndef RSPH_LANES_3D
#define RSPH_LANES_3D 4
#endif
template <int D>
struct Lanes;
template <>
struct Lanes<2> {
    static constexpr int G = RSPH_LANES_2D;
};
template <>
struct Lanes<3> {
    static constexpr int G = RSPH_LANES_3D;
};
// list entries per lane whose gathers are issued together in the pair passes
// (measured: 1 in 2D, where the lists are short; in 3D 4 with FP32 records
// and 2 with FP64 records, whose registers would otherwise cut occupancy)
#ifndef RSPH_CHUNK_2D
#define RSPH_CHUNK_2D 1
#endif
#ifndef RSPH_CHUNK_3D
#define RSPH_CHUNK_3D 4
#endif
template <typename R, int D>
struct Chunk {
    static constexpr int N = D == 2 ? RSPH_CHUNK_2D : (sizeof(R) == 4 ? RSPH_CHUNK_3D : 2);
};
// per-pass choices in 2D (the advection pass takes 2 in both dimensions)
#ifndef RSPH_CHUNK_2D_COLOUR
#define RSPH_CHUNK_2D_COLOUR RSPH_CHUNK_2D
#endif
#ifndef RSPH_CHUNK_2D_FORCE
#define RSPH_CHUNK_2D_FORCE RSPH_CHUNK_2D
#endif
#ifndef RSPH_CHUNK_2D_CONTINUITY
#define RSPH_CHUNK_2D_CONTINUITY RSPH_CHUNK_2D
#endif
#ifndef RSPH_CHUNK_2D_SHIFT
#define RSPH_CHUNK_2D_SHIFT RSPH_CHUNK_2D
#endif
#ifndef RSPH_CHUNK_2D_ADVECTION
#define RSPH_CHUNK_2D_ADVECTION 2
#endif
enum class Pass { Colour, Force, Continuity, Shift, Advection };
template <typename R, int D, Pass P>
struct PassChunk {
    static constexpr int N2 = P == Pass::Colour       ? RSPH_CHUNK_2D_COLOUR
                              : P == Pass::Force      ? RSPH_CHUNK_2D_FORCE
                              : P == Pass::Continuity ? RSPH_CHUNK_2D_CONTINUITY
                              : P == Pass::Shift      ? RSPH_CHUNK_2D_SHIFT
                                                      : RSPH_CHUNK_2D_ADVECTION;
    static constexpr int N = D == 2 ? N2 : (P == Pass::Advection ? 2 : Chunk<R, D>::N);
};
// at least 4 lanes: a 256-thread block then covers at most 64 slots, i.e. lies
// inside one system, which the per-block partial maxima rely on
static_assert(RSPH_LANES_2D >= 4 && RSPH_LANES_3D >= 4, "lanes per slot");
static_assert(RSPH_LANES_2D <= kMaxLanes && RSPH_LANES_3D <= kMaxLanes, "lanes per slot");

// slot of this thread's group and its lane g in the group (no memory access)
template <int G>
__device__ __forceinline__ int64_t group_slot(int& g)
{
    const int64_t t = logical_block() * kBlock + threadIdx.x;
    g = (int)(t & (G - 1));
    return t / G;
}

// system of slot i < A.P; the 64 / G slots of a wave lie in one 64-slot block,
// hence one system
__device__ __forceinline__ Slot lookup_slot(const DevArrays& A, int64_t i)
{
    Slot c;
    c.i = i;
    c.lane = false;
    const int s = system_of_wave(A, __builtin_amdgcn_readfirstlane((int)(i >> 6)));
    c.s = s;
    if (s < 0) return c;
    const SysConst& S = A.sc[s];
    c.lane = i < S.p_off + S.p_n;
    return c;
}

template <int G>
__device__ __forceinline__ Slot slot_of_group(const DevArrays& A, int& g)
{
    const int64_t i = group_slot<G>(g);
    if (i >= A.P) return Slot{i, -1, false};
    return lookup_slot(A, i);
}

// Neighbour-list walk of the pair passes, lane g of particle i's group
// taking entries g, g + G, ... in order, CH at a time: the records of a chunk
// are gathered together (load(slot)) and the indices of the next chunk are
// loaded while the current one is evaluated; body(entry, records) gets the
// whole list entry, cell differences included.  The first chunk's indices are requested by
// start(), which needs only the slot, so that their latency overlaps the
// system lookup; entries past the count hold stale values and are never used
// as addresses (a lane past the count reuses its group's first entry).
template <int G, int CH>
struct NbrList {
    static_assert(G * CH <= kKmax2, "first chunk inside every list");
    const uint32_t* list;
    uint32_t jn[CH];

    __device__ __forceinline__ void start(const DevArrays& A, int64_t i, int g)
    {
        list = A.nbr + ((i >> 6) * A.kmax) * kWave + (i & 63);
#pragma unroll
        for (int u = 0; u < CH; ++u) jn[u] = list[(int64_t)(g + u * G) * kWave];
    }

    template <typename Load, typename Body>
    __device__ __forceinline__ void run(int g, int cnt, Load&& load, Body&& body)
    {
        for (int k0 = g; k0 < cnt; k0 += G * CH) {
            uint32_t jb[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) jb[u] = k0 + u * G < cnt ? jn[u] : jn[0];
            decltype(load(0u)) rec[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) rec[u] = load(jb[u] & kNbrIndexMask);
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int k = k0 + (CH + u) * G;
                if (k < cnt) jn[u] = list[(int64_t)k * kWave];
            }
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (k0 + u * G < cnt) body(jb[u], rec[u]);
        }
    }
};

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v)
{
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The packed substep passes gather {v, p} per neighbour and recover the rest
// of its state from the pressure: rho = rho0 + p / c0^2 (Eq. 3 solved for the
// density) and V = m / rho with the fluid's one particle mass.  Both sides of
// a pair recover a particle's values from the same record, so a pair's terms
// stay antisymmetric.
template <typename R>
struct FromPressure {
    // scalars, not arrays: an array indexed by the phase is placed in LDS
    R rho0_k, rho0_l, m_k, m_l, inv_c0sq;
    __device__ __forceinline__ explicit FromPressure(const SysConst& S)
        : rho0_k((R)S.rho0[0]), rho0_l((R)S.rho0[1]), m_k((R)S.mphase[0]), m_l((R)S.mphase[1]),
          inv_c0sq((R)S.inv_c0sq)
    {
    }
    // density and mass of a particle of fluid ph (a wall's are never used);
    // the select is taken between values, not members (a select between the
    // members' addresses made the compiler keep them in an LDS table)
    __device__ __forceinline__ R rho(int ph, R p) const
    {
        const R a = rho0_l, b = rho0_k;
        return ((ph & 1) ? a : b) + p * inv_c0sq;
    }
    __device__ __forceinline__ R m(int ph) const
    {
        const R a = m_l, b = m_k;
        return (ph & 1) ? a : b;
    }
    // {rho, V, p, 0}
    __device__ __forceinline__ Q4<R> operator()(int ph, R p) const
    {
        const R r = rho(ph, p);
        return Q4<R>{r, m(ph) / r, p, R(0)};
    }
};

__device__ __forceinline__ bool substep_on(const SysDyn& D, int mode)
{
    return mode ? D.stepping != 0 : D.state == kSubstepping;
}

// ---------------------------------------------------------------------------
// binning: cell key, counting sort (histogram, scan, scatter), ordering of
// each cell by the caller's particle index, move of the state into that order
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Start of a launch cycle (step mode): systems that finished an advection
// step go back to the boundary, or to idle once their target is reached or
// after a fault; systems at the boundary with steps left run this cycle's
// prologue.  The new state depends only on fields no thread of the key pass
// writes (step count, target, health) and maps every state it can produce to
// itself, so each thread evaluates it for its own system and the system's
// first slot stores it: a thread that reads the stored state gets the same
// answer as one that reads the old state.
__device__ __forceinline__ int cycle_state(const SysDyn& D)
{
    const int st = D.state;
    if (st == kSubstepping) return st;
    const bool done = D.n_outer >= D.target || (D.health & ~kHealthClose);
    return done ? kIdle : kBoundary;
}

// Cell key of every particle of a stepping system, its rank among the
// particles of its cell in atomic order (one atomic per run of equal cells in
// a wave), and a snapshot of the state into the second buffer, from which the
// rank pass then moves it into sorted order.
template <int D>
__global__ __launch_bounds__(kBlock) void k_key(DevArrays A, int64_t group)
{
    const int64_t i = logical_block() * kBlock + threadIdx.x;
    if (i >= A.P) return;
    // loads that need only the slot, issued together
    double x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) {
        x[a] = A.pos[a][i];
        v[a] = A.vel[a][i];
    }
    const double rho = A.rho[i], drho = A.drho[i], mass = A.mass[i];
    const int32_t id = A.id[i], phase = A.phase[i];
    double xo[3];
    load_pos<D>(A, i, xo);  // position at the last binning
    const Slot c = lookup_slot(A, i);
    if (c.s < 0) return;  // wave-uniform: a wave lies in one system or in none
    SysDyn& Dy = A.sd[c.s];
    const SysConst& S = A.sc[c.s];
    // the system's state is the same for the whole wave, so these returns are
    // too; the wave's padding slots stay to the end (the shuffles below)
    if (A.mode == 0) {
        const int st = cycle_state(Dy);
        if (c.lane && c.i == S.p_off) {
            Dy.state = st;
            Dy.stepping = st == kBoundary;
            if (st == kBoundary && A.work) atomicOr(A.work + group, 1);
        }
        if (st != kBoundary) return;
    } else if (!Dy.stepping) {
        return;
    }
    const bool on = c.lane;
    uint32_t gkey = 0xffffffffu;  // global cell of the particle; none for padding
    if (on) {
        int ck[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            double xa = x[a];
            if (xa < 0.0) xa = __dadd_rn(xa, S.box[a]);
            if (xa >= S.box[a]) xa = __dsub_rn(xa, S.box[a]);
            A.pos2[a][i] = xa;
            A.vel2[a][i] = v[a];
            ck[a] = cell_of(xa, S, a);
        }
        A.rho2[i] = rho;
        A.drho2[i] = drho;
        A.mass2[i] = mass;
        A.id2[i] = id;
        A.phase2[i] = phase;
        const uint32_t key = (uint32_t)(ck[0] + S.ncell[0] * (ck[1] + S.ncell[1] * ck[2]));
        A.key[i] = key;
        gkey = (uint32_t)S.c_off + key;
        // the same slot held the same particle at the last binning: more than
        // one cell of motion since then (periodic distance) is counted, once
        // per advection step, when the step begins
        if (A.mode == 0 && Dy.binned) {
            bool far = false;
            for (int a = 0; a < D; ++a) {
                const int dc = abs(ck[a] - cell_of(xo[a], S, a));
                far |= dc > 1 && dc < S.ncell[a] - 1;
            }
            if (far) Dy.displaced = 1;
        }
    }
    // Ranks by runs: the slots are sorted by cell from the last binning, so
    // neighbouring lanes mostly share a cell.  The first lane of each run of
    // equal cells reserves the run's ranks with one atomic; every rank of a
    // cell is still taken exactly once.
    const int lane = threadIdx.x & 63;
    const uint32_t prev = __shfl_up(gkey, 1, 64);
    const bool lead = on && (lane == 0 || prev != gkey);
    const unsigned long long lm = __ballot(lead);
    const unsigned long long bm = __ballot(lead || !on);  // run boundaries
    int base = 0;
    if (lead) {
        const unsigned long long above = lane == 63 ? 0ull : bm & (~0ull << (lane + 1));
        const int next = above ? __ffsll((long long)above) - 1 : 64;
        base = atomicAdd(&A.cell_cnt[gkey], next - lane);
    }
    const unsigned long long upto = lm & (lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull));
    const int ld = upto ? 63 - __clzll((long long)upto) : lane;
    const int b = __shfl(base, ld, 64);
    if (on) A.rank[i] = b + (lane - ld);
}

// exclusive scan of cell_cnt[0..n) into cell_start[0..n], three phases
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int* lds, int& total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wv] = x;
    __syncthreads();
    int off = 0;
    for (int k = 0; k < wv; ++k) off += lds[k];
    total = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return off + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t* in, int64_t n, int32_t* part)
{
    __shared__ int lds[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = base + (int64_t)k * kBlock + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    int total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// single block: exclusive scan of the tile totals (at most kScanTile of them)
__global__ __launch_bounds__(kBlock) void k_scan_partials(int32_t* part, int64_t nparts)
{
    __shared__ int lds[4];
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = (int64_t)threadIdx.x * kScanItems + k;
        v[k] = idx < nparts ? part[idx] : 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, lds, total);
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = (int64_t)threadIdx.x * kScanItems + k;
        if (idx < nparts) part[idx] = ex;
        ex += v[k];
    }
}

// the final phase also clears the counts for the next histogram
__global__ __launch_bounds__(kBlock) void k_scan_final(int32_t* in, int64_t n, const int32_t* part,
                                                       int32_t* out)
{
    __shared__ int lds[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = base + k;
        v[k] = idx < n ? in[idx] : 0;
        if (idx < n) in[idx] = 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, lds, total) + part[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = base + k;
        if (idx < n) out[idx] = ex;
        ex += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = ex;
}

// scatter in arrival order (the cell-relative rank of the histogram atomics)
__global__ __launch_bounds__(kBlock) void k_scatter(DevArrays A)
{
    Slot c = slot_of(A);
    if (!c.lane) return;
    if (!A.sd[c.s].stepping) return;
    const SysConst& S = A.sc[c.s];
    const uint32_t key = A.key[c.i];
    const int64_t dest = S.p_off + (A.cell_start[S.c_off + key] - A.cell_start[S.c_off]) + A.rank[c.i];
    A.tmp[dest] = (int32_t)c.i;
}

// Grids of at most kScanSmall cells: every block of the scatter scans all the
// cell counts in LDS itself, in place of a scan pass; block 0 stores the cell
// starts for the passes that follow, and the rank pass clears the counts.
constexpr int kScanSmall = 8192;
constexpr int kScanSmallItems = kScanSmall / kBlock;
// LDS index of cell start k: one word of padding per 32, so that the threads'
// runs of 32 consecutive starts fall on different banks
__device__ __forceinline__ int64_t st_pad(int64_t k) { return k + (k >> 5); }

__global__ __launch_bounds__(kBlock) void k_scatter_small(DevArrays A, int64_t n)
{
    __shared__ int32_t st[kScanSmall + 1 + (kScanSmall + 1) / 32 + 1];
    __shared__ int lds[kBlock / kWave];
    // the slot's own loads first, so that their latency overlaps the scan
    const Slot c = slot_of(A);
    uint32_t key = 0;
    int32_t rk = 0;
    bool on = c.lane && A.sd[c.s].stepping;
    if (on) {
        key = A.key[c.i];
        rk = A.rank[c.i];
    }
    const int64_t base = (int64_t)threadIdx.x * kScanSmallItems;
    int v[kScanSmallItems];
    int sum = 0;
    // 16-byte loads where the thread's items lie below n (the counts are
    // 256-byte aligned and base is a multiple of 32)
    static_assert(kScanSmallItems % 4 == 0, "16-byte loads");
    for (int k = 0; k < kScanSmallItems; k += 4) {
        const int64_t idx = base + k;
        if (idx + 4 <= n) {
            const int4 q = *(const int4*)(A.cell_cnt + idx);
            v[k] = q.x;
            v[k + 1] = q.y;
            v[k + 2] = q.z;
            v[k + 3] = q.w;
        } else {
            for (int u = 0; u < 4; ++u) v[k + u] = idx + u < n ? A.cell_cnt[idx + u] : 0;
        }
    }
    for (int k = 0; k < kScanSmallItems; ++k) sum += v[k];
    int total;
    int ex = block_exclusive_scan(sum, lds, total);
    for (int k = 0; k < kScanSmallItems; ++k) {
        const int64_t idx = base + k;
        if (idx < n) st[st_pad(idx)] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) st[st_pad(n)] = total;
    __syncthreads();
    if (blockIdx.x == 0)
        for (int64_t k = threadIdx.x; k <= n; k += kBlock) A.cell_start[k] = st[st_pad(k)];
    if (!on) return;
    const SysConst& S = A.sc[c.s];
    const int64_t dest = S.p_off + (st[st_pad(S.c_off + key)] - st[st_pad(S.c_off)]) + rk;
    A.tmp[dest] = (int32_t)c.i;
}

// Final, canonical order: within its cell a particle's rank is the number of
// cell members before it in (x, caller index) order (ids are unique), so the
// sorted order is (cell, x, id) whatever order the atomics produced; the
// neighbour pass relies on each cell's members ascending in x.  Each particle then
// moves its state from the snapshot into its sorted slot of the primary arrays
// and writes its packed position record; the per-fluid |v| maxima of each 64
// source slots go to the partials of the advection time step.  On grids
// scanned inside the scatter this pass clears the cell counts (clear_n cells).
template <int D>
__global__ __launch_bounds__(kBlock) void k_rank(DevArrays A, int64_t clear_n)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < clear_n; k += (int64_t)gridDim.x * kBlock)
        A.cell_cnt[k] = 0;
    const int64_t i = logical_block() * kBlock + threadIdx.x;
    if (i >= A.P) return;
    // loads that need only the slot, issued together
    const uint32_t key = A.key[i];
    const int32_t me = A.id2[i];
    double x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) {
        x[a] = A.pos2[a][i];
        v[a] = A.vel2[a][i];
    }
    const double rho = A.rho2[i], drho = A.drho2[i], mass = A.mass2[i];
    const int ph = A.phase2[i];
    const Slot c = lookup_slot(A, i);
    if (c.s < 0) return;
    if (!A.sd[c.s].stepping) return;  // wave-uniform
    unsigned long long m0 = 0, m1 = 0;
    if (c.lane) {
        const SysConst& S = A.sc[c.s];
        const int64_t base = S.p_off - A.cell_start[S.c_off];
        const int64_t b = base + A.cell_start[S.c_off + key], e = base + A.cell_start[S.c_off + key + 1];
        // x compared through its bit pattern (x + 0 turns -0 into +0): for the
        // wrapped x >= 0 this is the numeric order, and it stays a strict
        // total order with the caller index whatever the values, so the ranks
        // of a cell are always a permutation
        const double* xs = A.pos2[0];
        const long long kme = __double_as_longlong(x[0] + 0.0);
        auto before = [&](int32_t t) {
            const long long kt = __double_as_longlong(xs[t] + 0.0);
            return (int)(kt < kme || (kt == kme && A.id2[t] < me));
        };
        int r = 0;
        // four members at a time, their loads in flight together
        int64_t k = b;
        for (; k + 4 <= e; k += 4) {
            const int32_t t0 = A.tmp[k], t1 = A.tmp[k + 1], t2 = A.tmp[k + 2], t3 = A.tmp[k + 3];
            r += before(t0) + before(t1) + before(t2) + before(t3);
        }
        for (; k < e; ++k) r += before(A.tmp[k]);
        const int64_t d = b + r;
        A.perm[d] = (int32_t)i;
        double v2 = 0.0;
        for (int a = 0; a < D; ++a) {
            A.pos[a][d] = x[a];
            A.vel[a][d] = v[a];
            v2 += v[a] * v[a];
        }
        store_pos<D>(A, d, x, ph);
        if constexpr (D == 3) store_xq(A, d, x, ph, S);
        A.rho[d] = rho;
        A.drho[d] = drho;
        A.mass[d] = mass;
        A.id[d] = me;
        A.phase[d] = ph;
        if (i == S.p_off) A.sd[c.s].binned = 1;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(sqrt(v2));
        if (ph == 0) m0 = bits;
        else if (ph == 1) m1 = bits;  // a wall's speed is not the fluids'
    }
    m0 = wave_max_u64(m0);
    m1 = wave_max_u64(m1);
    if ((threadIdx.x & 63) == 0) {
        const int64_t w = c.i >> 6;
        A.vpart[2 * w] = m0;
        A.vpart[2 * w + 1] = m1;
    }
}

// ---------------------------------------------------------------------------
// neighbour lists (frozen geometry of section 3.3), density summation, and the
// per-particle inputs of the pair loops
// ---------------------------------------------------------------------------

// Neighbour lists.  The candidates of one block's particles are staged in LDS:
// the block's 64 slots lie in a few consecutive cells of one or two cell rows,
// so the union of their 3^d stencils is at most two small boxes of cells whose
// particles are copied once per block as FP32 offsets (x from the box's x
// origin, y and z from their own cell corner).  A candidate is tested in FP32
// on these split positions.  Candidates within the FP32 error band of the
// cut-off (2h)^2 (at least a relative 1e-5) are decided on the spot by the
// exact FP64 predicate on the stored positions, so the neighbour set is
// exactly the one of the FP64 predicate.  The three cells of a stencil row
// are consecutive both in LDS and, unless the row wraps around the periodic
// box, in the cell-sorted slots, so a row is scanned as one range.
// The members of a cell ascend in x (the binning order), so a row's first and
// last cells are cut to the x sub-bins that reach within the cut-off: each
// staged cell holds, per edge of kXBins equal sub-bins, the first entry at or
// past that edge, and the entries cut off lie beyond the cut-off in x alone.
// Blocks whose union does not fit fall back to testing every candidate in FP64
// from global memory; both paths produce the same list in the same order
// (stencil cells in z, y, x order, slots ascending within a cell).
constexpr int kStageCells = 128;
constexpr int kStageCap = 2304;
constexpr int kXBins = 8;

// x edge s (0..kXBins) of the box-local x cell l: l w + s w / kXBins in FP32,
// one rounding per operation, so the staging and the candidate loop compute
// the same value
__device__ __forceinline__ float xbin_edge(int l, int s, float w, float ws)
{
    return __fadd_rn(__fmul_rn((float)l, w), __fmul_rn((float)s, ws));
}

// The union is kept as two boxes: one for the particles in the cell row
// (y, z) of the block's first particle, one for the rest.  A block that runs
// from the end of one row into the start of the next thus stages two compact
// boxes instead of one box as wide as the grid.
struct Stage {
    // x offset from its box's x origin (the lower corner of the box's first
    // x cell), y and z offsets from the candidate's own cell corner; w holds
    // the bits of -(box-local x cell << 26) (mod 2^32)
    float4 q[kStageCap];
    int32_t off[kStageCells + 1];  // LDS offset of each union cell (box 0's cells, then box 1's)
    int32_t gs[kStageCells];       // first global slot of each union cell
    // per union cell and x edge s: the first entry whose x offset is at or past
    // the edge (the cell's end if none)
    uint16_t xb[kStageCells * (kXBins + 1)];
    int32_t lo[2][3], hi[2][3];    // per box: cell-coordinate bounds of its particles
    int32_t dims[2][3];            // per box: extent (cells)
    int32_t ubase[2];              // per box: its first union cell
    int32_t row0;                  // cell row y + ny z of the block's first particle
    int32_t ok;
    int32_t wsum[kBlock / kWave];
};

__device__ __forceinline__ int wrap_cell(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// periodic image offset along axis a of the stencil cell c (unwrapped: one
// cell either way of the particle's own)
__device__ __forceinline__ double image_offset(const SysConst& S, int c, int a)
{
    return c < 0 ? -S.box[a] : (c >= S.ncell[a] ? S.box[a] : 0.0);
}

template <int D>
__device__ __forceinline__ int stage_union(const DevArrays& A, const SysConst& S, Stage& L, int64_t base,
                                           bool live, const int* ci, int g)
{
    const int t = threadIdx.x;
    if (t < 6) {
        L.lo[t / 3][t % 3] = 0x7fffffff;
        L.hi[t / 3][t % 3] = -0x7fffffff;
    }
    if (t == 0) L.row0 = 0x7fffffff;
    __syncthreads();
    const int row = ci[1] + S.ncell[1] * ci[2];
    if (live && g == 0) atomicMin(&L.row0, row);
    __syncthreads();
    const int box = row != L.row0;
    if (live && g == 0)
        for (int a = 0; a < D; ++a) {
            atomicMin(&L.lo[box][a], ci[a]);
            atomicMax(&L.hi[box][a], ci[a]);
        }
    __syncthreads();
    int ux[2], uy[2], uz[2], nb[2];
    for (int q = 0; q < 2; ++q) {
        const bool used = L.hi[q][0] >= L.lo[q][0];
        ux[q] = used ? L.hi[q][0] - L.lo[q][0] + 3 : 0;
        uy[q] = used ? L.hi[q][1] - L.lo[q][1] + 3 : 0;
        uz[q] = used ? (D == 3 ? L.hi[q][2] - L.lo[q][2] + 3 : 1) : 0;
        nb[q] = ux[q] * uy[q] * uz[q];
    }
    const int ncu = nb[0] + nb[1];
    // (the staged cell coordinate cx takes 23 bits)
    const bool fits_cells = nb[0] > 0 && ncu <= kStageCells && S.ncell[0] < (1 << 23);
    // per union cell (one thread each): its cell coordinates, count and first slot
    int cnt = 0, gs = 0, lx = 0, cx = 0, cy = 0, cz = 0;
    if (fits_cells && t < ncu) {
        const int q = t >= nb[0];
        const int u = t - (q ? nb[0] : 0);
        lx = u % ux[q];
        const int ly = (u / ux[q]) % uy[q], lz = u / (ux[q] * uy[q]);
        cx = wrap_cell(L.lo[q][0] - 1 + lx, S.ncell[0]);
        cy = wrap_cell(L.lo[q][1] - 1 + ly, S.ncell[1]);
        cz = D == 3 ? wrap_cell(L.lo[q][2] - 1 + lz, S.ncell[2]) : 0;
        const int64_t gc = S.c_off + cx + (int64_t)S.ncell[0] * (cy + (int64_t)S.ncell[1] * cz);
        const int a0 = A.cell_start[gc];
        cnt = A.cell_start[gc + 1] - a0;
        gs = (int)(base + a0);
    }
    // exclusive scan of the counts over the first 128 threads (two waves)
    const int lane = t & 63, wv = t >> 6;
    int x = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) L.wsum[wv] = x;
    __syncthreads();
    const int o0 = (wv == 0 ? 0 : L.wsum[0]) + x - cnt;
    const int total = L.wsum[0] + L.wsum[1];
    // lanes past the end of a range read up to 2 G - 1 entries beyond it
    const bool ok = fits_cells && total <= kStageCap - 2 * kMaxLanes;
    if (fits_cells && t < ncu) {
        L.off[t] = o0;
        L.gs[t] = gs;
    }
    // each cell's entries get their slot and cell coordinates, which the
    // entry pass below replaces by the staged record
    if (ok && t < ncu)
        for (int m = 0; m < cnt; ++m)
            L.q[o0 + m] = float4{__int_as_float(gs + m), __int_as_float(lx | (cx << 8)), __int_as_float(cy),
                                 __int_as_float(cz)};
    if (t == 0) {
        L.ok = ok;
        for (int q = 0; q < 2; ++q) {
            L.dims[q][0] = ux[q];
            L.dims[q][1] = uy[q];
            L.dims[q][2] = uz[q];
        }
        L.ubase[0] = 0;
        L.ubase[1] = nb[0];
        if (fits_cells) L.off[ncu] = total;
    }
    __syncthreads();
    if (!L.ok) return box;  // block-uniform
    for (int k = t; k < total; k += kBlock) {
        const float4 dsc = L.q[k];
        const int64_t j = __float_as_int(dsc.x);
        const int lxk = __float_as_int(dsc.y) & 0xff, cxk = __float_as_int(dsc.y) >> 8;
        double xj[3];
        load_pos<D>(A, j, xj);
        float4 c4;
        c4.x = (float)((double)lxk * S.cell[0] + (xj[0] - (double)cxk * S.cell[0]));
        c4.y = (float)(xj[1] - (double)__float_as_int(dsc.z) * S.cell[1]);
        c4.z = D == 3 ? (float)(xj[2] - (double)__float_as_int(dsc.w) * S.cell[2]) : 0.f;
        c4.w = __uint_as_float(0u - ((uint32_t)lxk << 26));
        L.q[k] = c4;
    }
    __syncthreads();
    // the sub-bin starts of each cell: a lower bound per x edge over the
    // cell's entries, which ascend in x (branch-free, the searches of one cell
    // interleaved)
    if (t < ncu) {
        const float w = (float)S.cell[0], ws = (float)(S.cell[0] / kXBins);
        const int e = o0 + cnt;
        float edge[kXBins + 1];
        int at[kXBins + 1];
#pragma unroll
        for (int sb = 0; sb <= kXBins; ++sb) {
            edge[sb] = xbin_edge(lx, sb, w, ws);
            at[sb] = o0;
        }
        if (cnt > 0) {
            int n = cnt;
            while (n > 1) {
                const int half = n >> 1;
#pragma unroll
                for (int sb = 0; sb <= kXBins; ++sb) at[sb] += L.q[at[sb] + half].x < edge[sb] ? half : 0;
                n -= half;
            }
#pragma unroll
            for (int sb = 0; sb <= kXBins; ++sb) at[sb] += L.q[at[sb]].x < edge[sb] ? 1 : 0;
        }
#pragma unroll
        for (int sb = 0; sb <= kXBins; ++sb) L.xb[t * (kXBins + 1) + sb] = (uint16_t)min(at[sb], e);
    }
    __syncthreads();
    return box;
}

// exact neighbour predicate: x_i - x_j, minus the periodic image offset of the
// stencil cell (the minimum image for every pair closer than 2h), squares
// summed in axis order, one rounding per operation
template <int D>
__device__ __forceinline__ double exact_r2(const DevArrays& A, const double* xi, int64_t j, double kx,
                                           double ky, double kz)
{
    // plain operators with contraction off: one rounding per operation (the
    // rounding-mode intrinsics alone do not keep the compiler from fusing a
    // product into the following sum)
#pragma clang fp contract(off)
    double xj[3];
    load_pos<D>(A, j, xj);
    double d = xi[0] - xj[0];
    if (kx != 0.0) d = d - kx;
    double r2 = d * d;
    d = xi[1] - xj[1];
    if (ky != 0.0) d = d - ky;
    r2 = r2 + d * d;
    if (D == 3) {
        d = xi[2] - xj[2];
        if (kz != 0.0) d = d - kz;
        r2 = r2 + d * d;
    }
    return r2;
}

// Ordered append of the hits of G consecutive candidates tested by the lanes
// of a group: the ballot keeps the list in candidate order.  entry() makes the
// list entry of a hit.
// The lists of a 64-slot range start at base (the same for every lane of a
// wave); entry e of the slot in lane position sl lies e * kWave + sl words
// after it.
struct ListOut {
    uint32_t* base;
    uint32_t sl;
    __device__ __forceinline__ void put(int at, uint32_t v) const
    {
        *(uint32_t*)((char*)base + (((uint32_t)at * kWave + sl) << 2)) = v;
    }
};

template <int G, typename Entry>
__device__ __forceinline__ void append_hits(bool hit, Entry&& entry, int gshift, uint32_t below, const ListOut& out,
                                            int kmax, int& cnt)
{
    const uint32_t gm = (uint32_t)(__builtin_amdgcn_ballot_w64(hit) >> gshift) & ((1u << G) - 1u);
    if (hit) {
        const int at = cnt + __popc(gm & below);
        if (at < kmax) out.put(at, entry());
    }
    cnt += __popc(gm);
}

// list entry: slot j and, per axis, the particle's cell minus the stencil
// cell's, plus one (the stencil offsets dx, dy, dz are -1, 0 or 1)
__device__ __forceinline__ uint32_t nbr_entry(int64_t j, int dx, int dy, int dz)
{
    return (uint32_t)j | ((uint32_t)(1 - dx) << 26) | ((uint32_t)(1 - dy) << 28) | ((uint32_t)(1 - dz) << 30);
}

// Every candidate of the 3^d stencil tested by the exact FP64 predicate on
// positions in global memory (blocks whose union does not fit in LDS).
template <int D, int G>
__device__ void scan_global(const DevArrays& A, const SysConst& S, int64_t i, const double* xi, const int* ci,
                            int ph, bool live, int g, int gshift, uint32_t below, int64_t base, const ListOut& out,
                            int& cnt)
{
    const int zr = D == 3 ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz) {
        int cz = ci[2] + dz;
        double kz = 0.0;
        if (D == 3) {
            if (cz < 0) { cz += S.ncell[2]; kz = -S.box[2]; }
            else if (cz >= S.ncell[2]) { cz -= S.ncell[2]; kz = S.box[2]; }
        }
        for (int dy = -1; dy <= 1; ++dy) {
            int cy = ci[1] + dy;
            double ky = 0.0;
            if (cy < 0) { cy += S.ncell[1]; ky = -S.box[1]; }
            else if (cy >= S.ncell[1]) { cy -= S.ncell[1]; ky = S.box[1]; }
            for (int dx = -1; dx <= 1; ++dx) {
                int cx = ci[0] + dx;
                double kx = 0.0;
                if (cx < 0) { cx += S.ncell[0]; kx = -S.box[0]; }
                else if (cx >= S.ncell[0]) { cx -= S.ncell[0]; kx = S.box[0]; }
                int64_t jb = 0, je = 0;
                if (live) {
                    const int64_t gc = S.c_off + cx + (int64_t)S.ncell[0] * (cy + (int64_t)S.ncell[1] * cz);
                    jb = base + A.cell_start[gc];
                    je = base + A.cell_start[gc + 1];
                }
                for (int64_t j0 = jb; j0 < je; j0 += G) {
                    const int64_t j = j0 + g;
                    bool hit = false;
                    if (j < je && j != i) {
                        hit = exact_r2<D>(A, xi, j, kx, ky, kz) < S.cut2;
                    }
                    append_hits<G>(hit, [&] { return nbr_entry(j, dx, dy, dz); }, gshift, below, out, A.kmax,
                                   cnt);
                }
            }
        }
    }
}

// Kernel sum sigma_i = W(0) + sum_j W_ij over particle i's list, the
// normalised density summation rho_i = rho0_i sigma_i / sigma0, and the
// {rho, V, p} record of the advection-step passes, and whether a neighbour is
// of the other phase (the interface flag, stored with the frozen geometry
// record); flags pairs closer than 1e-9 h.  FP64 in both forms: the density decides the pressure
// c0^2 (rho - rho0), which amplifies a density error by rho / (rho - rho0).
// Every lane of the group takes part; the lane that stores (lane 0 of a live
// slot) gets true and the volume V.
template <typename R, int D, int G>
__device__ __forceinline__ bool density_summation(const DevArrays& A, const SysConst& S, SysDyn& Dy, int64_t i,
                                                  int g, bool live, int cnt, const double* xi, double& V)
{
    const int ph = live ? A.phase[i] : 0;
    double wsum = 0.0;
    int coincident = 0, close = 0, cross = 0;
    // in 2D every lane's few entries are gathered at once
    constexpr int CH = D == 2 ? 4 : Chunk<R, D>::N;
    if constexpr (D == 3 && sizeof(R) == 4) {
        // mixed form: r_ij from the fixed-point offsets and the cell
        // difference of the list entry, (u_i - u_j - dx 2^31) cell / 2^31,
        // exact but for the one rounding of the product
        const U3* xq = (const U3*)A.xq;
        const U3 ui = xq[i];
        const double qc[3] = {S.cell[0] * 0x1p-31, S.cell[1] * 0x1p-31, S.cell[2] * 0x1p-31};
        for_neighbours<G, CH>(
            A, i, g, live ? cnt : 0, [&](uint32_t j) { return xq[j]; },
            [&](uint32_t e, const U3& q) {
                const int phj = (int)((q.x >> 31) | ((q.y >> 30) & 2u));
                cross |= phj != ph && phj != kWall;  // walls carry no colour
                const uint32_t f = e ^ 0x54000000u;
                const double rx = ((double)(int32_t)((ui.x & 0x7fffffffu) - (q.x & 0x7fffffffu)) -
                                   (double)((int32_t)(f << 4) >> 30) * 2147483648.0) * qc[0];
                const double ry = ((double)(int32_t)((ui.y & 0x7fffffffu) - (q.y & 0x7fffffffu)) -
                                   (double)((int32_t)(f << 2) >> 30) * 2147483648.0) * qc[1];
                const double rz = ((double)(int32_t)(ui.z - q.z) - (double)((int32_t)f >> 30) * 2147483648.0) *
                                  qc[2];
                const double r2 = rx * rx + ry * ry + rz * rz;
                // r to about 1e-13: the hardware reciprocal square root
                // (about 2^-22) and one Newton step, far inside the 1e-9 h of
                // the offsets; r = 0 (a flagged coincident pair) kept exact
                const double y0 = __builtin_amdgcn_rsq(r2);
                const double y1 = y0 * (1.5 - 0.5 * r2 * y0 * y0);
                const double r = r2 > 0.0 ? r2 * y1 : 0.0;
                wsum += wendland_w(r * S.inv_h, S.w_alpha);
                coincident |= r2 < S.coincident2;
                close |= r2 < S.close2;
            });
    } else
    for_neighbours<G, CH>(
        A, i, g, live ? cnt : 0,
        [&](uint32_t j) {
            Pos3 q;  // one record of D doubles per neighbour
            load_pos<D>(A, j, q.x, &q.ph);
            return q;
        },
        [&](uint32_t j, const Pos3& rj) {
            cross |= rj.ph != ph && rj.ph != kWall;  // walls carry no colour
            double r2 = 0.0;
            for (int a = 0; a < D; ++a) {
                double d = xi[a] - rj.x[a];
                if (d > S.half_box[a]) d -= S.box[a];
                else if (d < -S.half_box[a]) d += S.box[a];
                r2 += d * d;
            }
            wsum += wendland_w(sqrt(r2) * S.inv_h, S.w_alpha);
            coincident |= r2 < S.coincident2;
            close |= r2 < S.close2;
        });
    wsum = group_sum<G>(wsum);
    for (int o = 1; o < G; o <<= 1) {
        coincident |= __shfl_xor(coincident, o, 64);
        close |= __shfl_xor(close, o, 64);
        cross |= __shfl_xor(cross, o, 64);
    }
    if (!live || g != 0) return false;
    if (coincident) flag_health(Dy, kHealthCoincident);
    if (close) flag_health(Dy, kHealthClose);
    int ci[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) ci[a] = cell_of(xi[a], S, a);
    const bool wall = ph == kWall;
    const bool iface = cross && !wall;
    A.flags[i] = iface ? kFlagInterface : 0;
    Geo<R>::template store<D>(A.geo, i, xi, ph, iface, S, ci);
    const double sigma = S.w0 + wsum;
    double rho = A.rho[i];
    const double mass = A.mass[i];
    // a wall particle keeps its density; it has no pressure of its own
    if (A.mode == 0 && !(S.flags & kNoDensitySummation) && !wall) {
        rho = S.rho0[ph] * sigma / S.sigma0;
        A.rho[i] = rho;
    }
    if (A.mode == 1) A.r_sigma[i] = sigma;
    V = mass / rho;
    const double p = wall ? 0.0 : S.c0sq * (rho - S.rho0[ph]);
    ((Q4<R>*)A.th[1])[i] = Q4<R>{(R)rho, (R)V, (R)p, (R)0};
    return true;
}

// In 2D the neighbour pass ends with the density summation over the new list
// (after a block barrier, the entries written by the other lanes of the group
// visible): the list is short, and at small sizes a pass costs mostly its
// launch.  In 3D the summation is a pass of its own: it gathers some 75
// positions per particle, and the LDS staging of the neighbour pass holds that
// pass to 4 blocks per CU, half the occupancy the gather-bound sum runs at
// alone.
template <typename R, int D>
__global__ __launch_bounds__(kBlock) void k_neighbours(DevArrays A)
{
    // the candidates of a stencil row are tested G at a time by the lanes of
    // the particle's group; an ordered ballot keeps the list in candidate
    // order
    constexpr int G = Lanes<D>::G;
    __shared__ Stage L;
    int g;
    Slot c = slot_of_group<G>(A, g);
    if (c.s < 0) return;  // block-uniform: a block lies in one 64-slot range
    SysDyn& Dy = A.sd[c.s];
    if (!Dy.stepping) return;
    const SysConst& S = A.sc[c.s];
    const int64_t i = c.i;
    const bool live = c.lane;
    const int gshift = (threadIdx.x & 63) & ~(G - 1);
    const uint32_t below = (1u << g) - 1u;
    const int64_t base = S.p_off - A.cell_start[S.c_off];
    double xi[3] = {0.0, 0.0, 0.0}, vel_i[3] = {0.0, 0.0, 0.0};
    int ci[3] = {0, 0, 0};
    int ph = 0;
    if (live) {
        load_pos<D>(A, i, xi);
        for (int a = 0; a < D; ++a) {
            ci[a] = cell_of(xi[a], S, a);
            vel_i[a] = A.vel[a][i];
        }
        ph = A.phase[i];
    }
    const int box = stage_union<D>(A, S, L, base, live, ci, g);
    int cnt = 0;
    // a wave's slots lie in one 64-slot range (64 / G of them), whose lists
    // start at a wave-uniform address
    const int64_t range = __builtin_amdgcn_readfirstlane((int)(i >> 6));
    const ListOut out{A.nbr + (range * A.kmax) * kWave, (uint32_t)(i & 63)};
    if (L.ok) {  // block-uniform
        float oi[3] = {0.f, 0.f, 0.f}, cellf[3];
        for (int a = 0; a < 3; ++a) {
            cellf[a] = (float)S.cell[a];
            if (a < D) oi[a] = (float)(xi[a] - (double)ci[a] * S.cell[a]);
        }
        const int i32 = (int)i;
        // the particle's cell, local to its box
        const int lx = ci[0] - L.lo[box][0] + 1, ly = ci[1] - L.lo[box][1] + 1;
        const int lz = D == 3 ? ci[2] - L.lo[box][2] + 1 : 0;
        // x offsets from the box's x origin: each rounds to within 2^-24 X of
        // its value, X the box's width, so the FP32 r^2 of a pair is within
        // (2^-23 X / h + 2^-22) (2h)^2 of the FP64 one; candidates within three
        // times that (at least 1e-5) of the cut-off take the exact test
        const float xo = (float)((double)lx * S.cell[0] + (xi[0] - (double)ci[0] * S.cell[0]));
        const double band =
            fmax(1e-5, 3.0 * (ldexp((double)L.dims[box][0] * S.cell[0] * S.inv_h, -23) + ldexp(1.0, -22)));
        const float cut_hi = (float)(S.cut2 * (1.0 + band)), cut_lo = (float)(S.cut2 * (1.0 - band));
        // The sub-bins of a row's first and last cells that the particle
        // reaches: an entry left of the first cell's edge s_lo - 1 has x offset
        // below xo - reach, one at or right of the last cell's edge s_hi above
        // xo + reach.  With reach = sqrt(cut_hi) (1 + 2^-12) either has
        // fl(ax^2) >= cut_hi, and so r^2 in FP32 as well (every rounding of a
        // sum of squares is monotone): the FP32 test rejects it.
        const float w = cellf[0], ws = (float)(S.cell[0] / kXBins);
        const float reach = sqrtf(cut_hi) * (1.f + 0x1p-12f);
        const float lo_x = xo - reach, hi_x = xo + reach;
        int s_lo = 0, s_hi = 0;
        for (int sb = 0; sb <= kXBins; ++sb) {
            s_lo += xbin_edge(lx - 1, sb, w, ws) <= lo_x;
            s_hi += xbin_edge(lx + 1, sb, w, ws) <= hi_x;
        }
        const int zr = D == 3 ? 1 : 0;
        for (int dz = -zr; dz <= zr; ++dz) {
            const float rz0 = oi[2] - (float)dz * cellf[2];
            const double kz = D == 3 ? image_offset(S, ci[2] + dz, 2) : 0.0;
            for (int dy = -1; dy <= 1; ++dy) {
                const float ry0 = oi[1] - (float)dy * cellf[1];
                const double ky = image_offset(S, ci[1] + dy, 1);
                // the row's three cells, the first and last cut to the
                // particle's reach in x
                int u0 = 0, rb = 0, re = 0;
                bool contiguous = true;
                if (live) {
                    u0 = L.ubase[box] + (lx - 1) + L.dims[box][0] * ((ly + dy) + L.dims[box][1] * (lz + dz));
                    rb = s_lo == 0 ? L.off[u0] : (int)L.xb[u0 * (kXBins + 1) + s_lo - 1];
                    re = s_hi > kXBins ? L.off[u0 + 3] : (int)L.xb[(u0 + 2) * (kXBins + 1) + s_hi];
                    contiguous = L.gs[u0 + 1] - L.gs[u0] == L.off[u0 + 1] - L.off[u0] &&
                                 L.gs[u0 + 2] - L.gs[u0 + 1] == L.off[u0 + 2] - L.off[u0 + 1];
                }
                // a row that wraps around the box is scanned cell by cell
                const int nseg = contiguous ? 1 : 3;
                for (int sgm = 0; sgm < nseg; ++sgm) {
                    const int kb = contiguous || sgm == 0 ? rb : L.off[u0 + sgm];
                    const int ke = contiguous || sgm == 2 ? re : L.off[u0 + sgm + 1];
                    // slots fit in 32 bits (the slot capacity is checked on the host)
                    const int uc = contiguous ? u0 : u0 + sgm;
                    const int jofs = L.gs[uc] - L.off[uc];
                    const int kself = i32 - jofs;  // the particle itself: slot jofs + k == i
                    // The list entry of candidate k is k + ebase + q.w (mod 2^32):
                    // jofs + k is the slot, and (1 + lx) << 26 plus the staged
                    // -(lx_j << 26) is (1 - dx) << 26 with dx = lx_j - lx in
                    // {-1, 0, 1}, as nbr_entry lays the entry out.
                    const uint32_t ebase = (uint32_t)jofs + ((uint32_t)(1 + lx) << 26) +
                                           ((uint32_t)(1 - dy) << 28) + ((uint32_t)(1 - dz) << 30);
                    // two entries per lane and iteration; lanes past the range
                    // read entries beyond it (inside the staging array) and
                    // discard them
                    auto test = [&](int k, const float4& q) {
                        const float ax = xo - q.x;
                        const float ay = ry0 - q.y;
                        const float az = D == 3 ? rz0 - q.z : 0.f;
                        const float r2f = ax * ax + ay * ay + az * az;
                        const uint32_t qw = __float_as_uint(q.w);
                        // (no short circuit: one mask, no branch)
                        bool hit = (k < ke) & (k != kself) & (r2f < cut_hi);
                        if (hit && r2f >= cut_lo) {  // within the FP32 error of the cut-off
                            // the stencil x offset of the candidate's cell
                            const int dx = (int)((0u - qw) - ((uint32_t)lx << 26)) >> 26;
                            hit = exact_r2<D>(A, xi, jofs + k, image_offset(S, ci[0] + dx, 0), ky, kz) < S.cut2;
                        }
                        append_hits<G>(hit, [&] { return (uint32_t)k + ebase + qw; }, gshift, below, out, A.kmax,
                                       cnt);
                    };
                    for (int k0 = kb; k0 < ke; k0 += 2 * G) {
                        const int ka = k0 + g, kc = k0 + G + g;
                        const float4 qa = L.q[ka];
                        const float4 qc = L.q[kc];
                        test(ka, qa);
                        test(kc, qc);
                    }
                }
            }
        }
    } else {
        scan_global<D, G>(A, S, i, xi, ci, ph, live, g, gshift, below, base, out, cnt);
    }
    if (cnt > A.kmax) {  // group-uniform
        if (live && g == 0) flag_health(Dy, kHealthNeighbours);
        cnt = A.kmax;
    }
    double V = 0.0;
    bool store = live && g == 0;
    if constexpr (D == 2) {
        __syncthreads();
        store = density_summation<R, D, G>(A, S, Dy, i, g, live, cnt, xi, V);
    }
    if (!store) return;
    A.ncount[i] = cnt;
    if (A.mode == 1)
        for (int a = 0; a < 3; ++a) A.r_gradc[3 * i + a] = 0.0;  // interface particles overwrite
    // the volume rides in the spare component of the velocity record read by
    // the advection pass (in 3D stored by the density pass)
    ((Q4<R>*)A.vbuf[0])[i] = Q4<R>{(R)vel_i[0], (R)vel_i[1], (R)vel_i[2], (R)V};
    ((Q4<R>*)A.col)[i] = Q4<R>{(R)0, (R)0, (R)0, (R)0};
}

// the density summation as a pass of its own (3D)
template <typename R, int D>
__global__ __launch_bounds__(kBlock) void k_density(DevArrays A)
{
    constexpr int G = Lanes<D>::G;
    int g;
    Slot c = slot_of_group<G>(A, g);
    if (c.s < 0) return;
    SysDyn& Dy = A.sd[c.s];
    if (!Dy.stepping) return;
    const SysConst& S = A.sc[c.s];
    const int64_t i = c.i;
    double xi[3] = {0.0, 0.0, 0.0};
    int cnt = 0;
    if (c.lane) {
        for (int a = 0; a < D; ++a) xi[a] = A.pos[a][i];
        cnt = A.ncount[i];
    }
    double V = 0.0;
    if (density_summation<R, D, G>(A, S, Dy, i, g, c.lane, cnt, xi, V))
        reinterpret_cast<R*>((Q4<R>*)A.vbuf[0] + i)[3] = (R)V;
}

// ---------------------------------------------------------------------------
// advection-step pair pass 1: viscous acceleration (Eq. 13), correction matrix
// (Eq. 15), near-interface flag
// ---------------------------------------------------------------------------

__device__ void begin_advection_step(const DevArrays& A, const SysConst& S, SysDyn& D);

template <typename R, int D>
__global__ __launch_bounds__(kBlock) void k_advection(DevArrays A)
{
    constexpr int G = Lanes<D>::G;
    int g;
    const int64_t i = group_slot<G>(g);
    if (i >= A.P) return;
    // loads that need only the slot, issued together
    using GT = typename GeoT<R, D>::T;
    const GT* geo = (const GT*)A.geo;
    const Q4<R>* th = (const Q4<R>*)A.th[1];
    const Q4<R>* vb = (const Q4<R>*)A.vbuf[0];
    NbrList<G, PassChunk<R, D, Pass::Advection>::N> nl;
    nl.start(A, i, g);
    const GT gi_i = geo[i];
    const Q4<R> vi_i = vb[i];
    const int cnt_i = A.ncount[i];
    const Slot c = lookup_slot(A, i);
    if (c.s < 0) return;
    SysDyn& Dy = A.sd[c.s];
    if (!Dy.stepping) return;  // block-uniform
    const SysConst& S = A.sc[c.s];
    // the system's first block also sets the advection step (Eqs. 16, 18) from
    // the per-wave |v| maxima of the rank pass; no pass of this kernel reads the
    // fields it writes
    if (A.mode == 0 && logical_block() * (kBlock / G) == S.p_off) begin_advection_step(A, S, Dy);
    R cellr[3] = {(R)S.cell[0], (R)S.cell[1], (R)S.cell[2]};
    const R inv_h = (R)S.inv_h, coef = (R)S.dw_coef;
    R av[3] = {0, 0, 0};
    R M[6] = {0, 0, 0, 0, 0, 0};  // 00 01 02 11 12 22
    R u[3] = {0, 0, 0};           // sum_j W'_ij V_j r_ij / r, for the shift's B_i term
    int near = 0;
    GT gi{};
    Q4<R> vi{0, 0, 0, 0};
    int cnt = 0, phi = 0;
    if (c.lane) {
        gi = gi_i;
        vi = vi_i;
        phi = Geo<R>::phase(gi);
        cnt = cnt_i;
    }
    const bool wall_i = phi == kWall;  // a wall particle: its B only
    // the harmonic mean of Eq. 13 takes two values: eta_i within the fluid
    // (and against a wall), 2 eta_i eta_o / (eta_i + eta_o) across
    const R eta_i = (R)(phi ? S.eta[1] : S.eta[0]);
    const R eta_o = (R)(phi ? S.eta[0] : S.eta[1]);
    const R eta_x = eta_i + eta_o > R(0) ? R(2) * eta_i * eta_o / (eta_i + eta_o) : R(0);
    nl.run(
        g, cnt, [&](uint32_t j) { return GRecs<GT, R, 1>{geo[j], {vb[j]}}; },
        [&](uint32_t ent, const GRecs<GT, R, 1>& rj) {
            const GT gj = rj.g;
            R r[3];
            Geo<R>::template rij<D>(gi, gj, ent, S, cellr, r);
            const R r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const R inv_r = rsqrt_dist<R>(r2);
            const R dW = wendland_dw<R>(r2 * inv_r * inv_h, coef);
            const Q4<R> vj = rj.q[0];
            const R Vj = vj.w;  // volume, stored beside the velocity
            // a wall neighbour: the fluid's own viscosity against the wall's
            // velocity, with the mirror's volume V_i
            const int phj = Geo<R>::phase(gj);
            const bool wall_j = phj == kWall;
            const R eta_bar = (phj == phi || wall_j) ? eta_i : eta_x;
            const R f = wall_i ? R(0) : eta_bar * dW * inv_r * (wall_j ? vi.w : Vj);
            av[0] += f * (vi.x - vj.x);
            av[1] += f * (vi.y - vj.y);
            if (D == 3) av[2] += f * (vi.z - vj.z);
            const R gg = dW * Vj * inv_r;
            u[0] += gg * r[0];
            u[1] += gg * r[1];
            if (D == 3) u[2] += gg * r[2];
            M[0] += gg * r[0] * r[0];
            M[1] += gg * r[0] * r[1];
            M[3] += gg * r[1] * r[1];
            if (D == 3) {
                M[2] += gg * r[0] * r[2];
                M[4] += gg * r[1] * r[2];
                M[5] += gg * r[2] * r[2];
            }
            near |= Geo<R>::interface(gj);
        });
    for (int a = 0; a < D; ++a) {
        av[a] = group_sum<G>(av[a]);
        u[a] = group_sum<G>(u[a]);
    }
    M[0] = group_sum<G>(M[0]);
    M[1] = group_sum<G>(M[1]);
    M[3] = group_sum<G>(M[3]);
    if (D == 3) {
        M[2] = group_sum<G>(M[2]);
        M[4] = group_sum<G>(M[4]);
        M[5] = group_sum<G>(M[5]);
    }
    for (int o = 1; o < G; o <<= 1) near |= __shfl_xor(near, o, 64);
    if (!c.lane || g != 0) return;
    const R two_over_rho = R(2) / th[i].x;
    Q4<R> a4{two_over_rho * av[0], two_over_rho * av[1], two_over_rho * av[2], (R)0};
    ((Q4<R>*)A.av)[i] = a4;
    // B = -M^{-1} (M is symmetric)
    R B[6];
    if (D == 2) {
        const R det = M[0] * M[3] - M[1] * M[1];
        if (det != R(0) && isfinite((double)det)) {
            B[0] = -M[3] / det;
            B[1] = M[1] / det;
            B[3] = -M[0] / det;
        } else {
            B[0] = R(1);
            B[1] = R(0);
            B[3] = R(1);
        }
        B[2] = B[4] = R(0);
        B[5] = R(0);
    } else {
        const R c00 = M[3] * M[5] - M[4] * M[4];
        const R c01 = M[2] * M[4] - M[1] * M[5];
        const R c02 = M[1] * M[4] - M[2] * M[3];
        const R c11 = M[0] * M[5] - M[2] * M[2];
        const R c12 = M[1] * M[2] - M[0] * M[4];
        const R c22 = M[0] * M[3] - M[1] * M[1];
        const R det = M[0] * c00 + M[1] * c01 + M[2] * c02;
        if (det != R(0) && isfinite((double)det)) {
            const R sc = R(-1) / det;
            B[0] = sc * c00;
            B[1] = sc * c01;
            B[2] = sc * c02;
            B[3] = sc * c11;
            B[4] = sc * c12;
            B[5] = sc * c22;
        } else {
            B[0] = B[3] = B[5] = R(1);
            B[1] = B[2] = B[4] = R(0);
        }
    }
    // the shift pass's records: sum_j (B_i + B_j) W'_ij V_j r_ij / r splits into
    // B_i u_i, this particle's own term, and sum_j W'_ij (V_j B_j) r_ij / r, which
    // takes V B of each neighbour beside its frozen offsets: 9 values in 3D
    // (two 16-byte records and one scalar), 5 in 2D (one record and a scalar)
    const R Vi = th[i].y;
    R VB[6];
    for (int q = 0; q < 6; ++q) VB[q] = Vi * B[q];
    Q4<R> t4;
    t4.x = B[0] * u[0] + B[1] * u[1] + B[2] * u[2];
    t4.y = B[1] * u[0] + B[3] * u[1] + B[4] * u[2];
    t4.z = B[2] * u[0] + B[4] * u[1] + B[5] * u[2];
    t4.w = (R)0;
    ((Q4<R>*)A.bt)[i] = t4;
    if (D == 3) {
        ((Q4<R>*)A.bm[0])[i] = Q4<R>{gi_i.x, gi_i.y, gi_i.z, VB[0]};
        ((Q4<R>*)A.bm[1])[i] = Q4<R>{VB[1], VB[2], VB[3], VB[4]};
        ((R*)A.bs)[i] = VB[5];
    } else {
        ((Q4<R>*)A.bm[0])[i] = Q4<R>{gi_i.x, gi_i.y, VB[0], VB[1]};
        ((R*)A.bs)[i] = VB[3];
    }
    A.flags[i] = (A.flags[i] & kFlagInterface) | (near ? kFlagNearInterface : 0);
    if (A.mode == 1) {
        for (int a = 0; a < 3; ++a) A.r_accv[3 * i + a] = a < D ? (double)(&a4.x)[a] : 0.0;
        const R full[9] = {B[0], B[1], B[2], B[1], B[3], B[4], B[2], B[4], B[5]};
        for (int q = 0; q < 9; ++q) A.r_b[9 * i + q] = 0.0;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) A.r_b[9 * i + a * D + b] = (double)full[a * 3 + b];
    }
}

// ---------------------------------------------------------------------------
// advection-step pair pass 2: position correction (Eq. 14), then the first
// half-step of substep 0 (density, pressure by Eq. 3, position)
// ---------------------------------------------------------------------------

template <typename R>
struct ShiftRec {
    Q4<R> q0, q1;  // {offsets, V B 00} and {V B 01 02 11 12} (3D); {offsets, V B 00 01} (2D)
    R z;           // V B 22 (3D), V B 11 (2D)
};

template <typename R, int D>
__global__ __launch_bounds__(kBlock) void k_shift(DevArrays A)
{
    constexpr int G = Lanes<D>::G;
    int g;
    const int64_t i = group_slot<G>(g);
    if (i >= A.P) return;
    // loads that need only the slot, issued together
    const Q4<R>* th = (const Q4<R>*)A.th[1];
    const Q4<R>* b0 = (const Q4<R>*)A.bm[0];
    const Q4<R>* b1 = (const Q4<R>*)A.bm[1];
    const R* bz = (const R*)A.bs;
    NbrList<G, PassChunk<R, D, Pass::Shift>::N> nl;
    nl.start(A, i, g);
    const Q4<R> gi_i = b0[i], t_i = ((const Q4<R>*)A.bt)[i];
    const int cnt_i = A.ncount[i];
    const Slot c = lookup_slot(A, i);
    if (c.s < 0) return;
    SysDyn& Dy = A.sd[c.s];
    if (!Dy.stepping) return;
    const SysConst& S = A.sc[c.s];
    R cellr[3] = {(R)S.cell[0], (R)S.cell[1], (R)S.cell[2]};
    const R inv_h = (R)S.inv_h, coef = (R)S.dw_coef;
    Q4<R> gi{0, 0, 0, 0};
    int cnt = 0;
    if (c.lane) {
        gi = gi_i;
        cnt = cnt_i;
    }
    R s[3] = {0, 0, 0};
    nl.run(
        g, cnt,
        [&](uint32_t j) {
            ShiftRec<R> q;
            q.q0 = b0[j];
            q.q1 = D == 3 ? b1[j] : Q4<R>{0, 0, 0, 0};
            q.z = bz[j];
            return q;
        },
        [&](uint32_t ent, const ShiftRec<R>& rj) {
            R r[3];
            Geo<R>::template rij<D>(gi, rj.q0, ent, S, cellr, r);
            const R r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const R inv_r = rsqrt_dist<R>(r2);
            const R f = wendland_dw<R>(r2 * inv_r * inv_h, coef) * inv_r;  // dW / r
            // (V_j B_j) r_ij, symmetric storage 00 01 02 11 12 22
            if (D == 2) {
                const R m00 = rj.q0.z, m01 = rj.q0.w, m11 = rj.z;
                s[0] += f * (m00 * r[0] + m01 * r[1]);
                s[1] += f * (m01 * r[0] + m11 * r[1]);
            } else {
                const R m00 = rj.q0.w, m01 = rj.q1.x, m02 = rj.q1.y, m11 = rj.q1.z, m12 = rj.q1.w, m22 = rj.z;
                s[0] += f * (m00 * r[0] + m01 * r[1] + m02 * r[2]);
                s[1] += f * (m01 * r[0] + m11 * r[1] + m12 * r[2]);
                s[2] += f * (m02 * r[0] + m12 * r[1] + m22 * r[2]);
            }
        });
    s[0] = t_i.x + group_sum<G>(s[0]);
    s[1] = t_i.y + group_sum<G>(s[1]);
    if (D == 3) s[2] = t_i.z + group_sum<G>(s[2]);
    if (!c.lane || g != 0) return;
    const int ph = A.phase[i];
    const bool wall = ph == kWall;
    double dr[3];
    for (int a = 0; a < 3; ++a) dr[a] = (a < D && !wall) ? -S.alpha_h2 * (double)s[a] : 0.0;
    Q4<R>* th0 = (Q4<R>*)A.th[0];
    // the packed substep passes take the pressure beside the velocity
    R* p_rec = reinterpret_cast<R*>((Q4<R>*)A.vbuf[0] + i) + 3;
    if (A.mode == 1 || wall) {  // a wall particle never moves and keeps its density
        if (A.mode == 1)
            for (int a = 0; a < 3; ++a) A.r_dr[3 * i + a] = dr[a];
        if (A.packed) *p_rec = th[i].z;
        else th0[i] = th[i];
        return;
    }
    if (!(S.flags & kNoShift))
        for (int a = 0; a < D; ++a) A.pos[a][i] += dr[a];
    // first half of substep 0
    const double dt = Dy.dt[0];
    const double rho = A.rho[i] + 0.5 * dt * A.drho[i];
    for (int a = 0; a < D; ++a) A.pos[a][i] += 0.5 * dt * A.vel[a][i];
    A.rho[i] = rho;
    const R p = (R)(S.c0sq * (rho - S.rho0[ph]));
    if (A.packed) *p_rec = p;
    else th0[i] = Q4<R>{(R)rho, (R)(A.mass[i] / rho), p, (R)0};
}

// ---------------------------------------------------------------------------
// advection-step state machine and time steps (Eqs. 16-18): one thread per
// system
// ---------------------------------------------------------------------------

__device__ __forceinline__ double dt_acoustic(const SysConst& S, const double* vmax)
{
    double dt = INFINITY;
    for (int f = 0; f < 2; ++f)
        dt = fmin(dt, fmin(S.cfl_ac * (S.h / (S.c0 + vmax[f])), S.dtac_surf[f]));
    return dt;
}

__device__ __forceinline__ bool dt_collapsed(const SysConst& S, double dt_ac)
{
    return !(dt_ac > 1e-12 * S.cfl_ac * S.h * S.inv_c0);
}

__global__ void k_set_stepping(DevArrays A, const int32_t* mask)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < A.nsys) A.sd[s].stepping = mask[s];
}

__global__ void k_set_targets(DevArrays A, const long long* targets)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < A.nsys && targets[s] >= 0) A.sd[s].target = targets[s];
}

// U partials per thread: entries e0 + t + u * 256 of the system's range
template <int U>
struct VParts {
    ulonglong2 v[U];
};

template <int U>
__device__ __forceinline__ void vmax_load(const DevArrays& A, int64_t e, int64_t e1, VParts<U>& p)
{
    const ulonglong2* vp = (const ulonglong2*)A.vpart;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = e + (int64_t)u * kBlock;
        p.v[u] = k < e1 ? vp[k] : make_ulonglong2(0ull, 0ull);
    }
}

template <int U>
__device__ __forceinline__ void vmax_fold(const VParts<U>& p, unsigned long long& m0, unsigned long long& m1)
{
#pragma unroll
    for (int u = 0; u < U; ++u) {
        m0 = p.v[u].x > m0 ? p.v[u].x : m0;
        m1 = p.v[u].y > m1 ? p.v[u].y : m1;
    }
}

// block maximum of the threads' values; identical in every lane, so held in
// scalar registers
__device__ __forceinline__ void vmax_block(unsigned long long m0, unsigned long long m1, unsigned long long* m)
{
    __shared__ unsigned long long red[2 * (kBlock / kWave)];
    m0 = wave_max_u64(m0);
    m1 = wave_max_u64(m1);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[2 * wv] = m0;
        red[2 * wv + 1] = m1;
    }
    __syncthreads();
    for (int k = 0; k < kBlock / kWave; ++k) {
        m0 = red[2 * k] > m0 ? red[2 * k] : m0;
        m1 = red[2 * k + 1] > m1 ? red[2 * k + 1] : m1;
    }
    m[0] = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(m0 >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)m0);
    m[1] = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(m1 >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)m1);
}

// first and one-past-last partial entry of a system
__device__ __forceinline__ void vmax_range(const SysConst& S, int64_t slots_per_entry, int64_t& e0, int64_t& e1)
{
    e0 = S.p_off / slots_per_entry;
    e1 = (S.p_off + ((S.p_n + kWave - 1) / kWave) * kWave) / slots_per_entry;
}

// Per-fluid maxima of |v| over one system from its partials, one entry per
// `slots_per_entry` slots (64 for the per-wave partials of the rank pass, 256 / G
// for the per-block partials of the force pass), as FP64 bit patterns: |v| is
// non-negative, so their integer order is the numeric one, and a non-finite
// |v| compares above every finite one.  Every thread of the 256-thread block
// takes part and gets the result; U partials per thread are in flight at a
// time.
template <int U>
__device__ __forceinline__ void reduce_vmax_bits(const DevArrays& A, const SysConst& S, int64_t slots_per_entry,
                                                 unsigned long long* m)
{
    int64_t e0, e1;
    vmax_range(S, slots_per_entry, e0, e1);
    unsigned long long m0 = 0, m1 = 0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += U * kBlock) {
        VParts<U> p;
        vmax_load<U>(A, e, e1, p);
        vmax_fold<U>(p, m0, m1);
    }
    vmax_block(m0, m1, m);
}

template <int U>
__device__ __forceinline__ void reduce_vmax(const DevArrays& A, const SysConst& S, int64_t slots_per_entry,
                                            double* vmax)
{
    unsigned long long m[2];
    reduce_vmax_bits<U>(A, S, slots_per_entry, m);
    vmax[0] = __longlong_as_double((long long)m[0]);
    vmax[1] = __longlong_as_double((long long)m[1]);
}

// start of an advection step: per-fluid max |v| over the system, the advection
// step (Eqs. 16, 18) and the first acoustic step (Eqs. 17, 18); called by every
// thread of one block of the system
__device__ void begin_advection_step(const DevArrays& A, const SysConst& S, SysDyn& D)
{
    double vmax[2];
    reduce_vmax<4>(A, S, kWave, vmax);
    if (threadIdx.x != 0) return;
    D.vmax[0] = vmax[0];
    D.vmax[1] = vmax[1];
    double dt_ad = INFINITY;
    for (int f = 0; f < 2; ++f) {
        double a = vmax[f] > 0.0 ? S.h / vmax[f] : INFINITY;
        dt_ad = fmin(dt_ad, fmin(S.cfl_ad * a, S.dtad_visc[f]));
    }
    const double dt_ac = dt_acoustic(S, vmax);
    // no motion and no viscosity: one acoustic step spans the advection step
    if (!isfinite(dt_ad)) dt_ad = dt_ac;
    D.dt_ad = dt_ad;
    D.tau = 0.0;
    D.ksub = 0;
    D.dt[0] = fmin(dt_ac, dt_ad);
    D.state = kSubstepping;
    if (D.displaced) {
        D.n_displaced += 1;
        D.displaced = 0;
    }
    if (dt_collapsed(S, dt_ac) || !(dt_ad > 0.0)) {
        atomicOr(&D.health, kHealthDtCollapse);
        D.state = kIdle;
    }
}

// End of substep k of an advection step: the clock advances by the substep's
// acoustic step; the next one follows from the per-fluid |v| maxima of the
// substep's velocity update (Eqs. 17, 18), clipped so that the advection step
// ends exactly at its length, unless that length is reached, the acoustic step
// collapsed or a velocity is not finite.
struct SubstepEnd {
    double tau;      // time into the advection step after substep k
    double dt_next;  // acoustic step of substep k + 1
    bool next;       // substep k + 1 follows
    bool collapse;
};

__device__ __forceinline__ SubstepEnd end_substep(const SysConst& S, double dt_ad, double tau, double dt,
                                                  uint32_t health, const double* vmax)
{
    SubstepEnd e;
    e.tau = tau + dt;
    const double dt_ac = dt_acoustic(S, vmax);
    e.collapse = dt_collapsed(S, dt_ac) || (health & kHealthNonFinite) || !isfinite(vmax[0]) ||
                 !isfinite(vmax[1]);
    e.next = !e.collapse && e.tau < dt_ad * (1.0 - 1e-12);
    e.dt_next = e.next ? fmin(dt_ac, dt_ad - e.tau) : 0.0;
    return e;
}

// stores the end of substep k (one thread per system)
__device__ __forceinline__ void commit_substep(SysDyn& D, long long k, double dt, const double* vmax,
                                               const SubstepEnd& e, int32_t end_state)
{
    D.tau = e.tau;
    D.t += dt;
    D.n_sub += 1;
    D.ksub = k + 1;
    D.dt_last = dt;
    D.vmax[0] = vmax[0];
    D.vmax[1] = vmax[1];
    if (e.next) {
        D.dt[(k + 1) & 1] = e.dt_next;
        return;
    }
    if (e.collapse) atomicOr(&D.health, kHealthDtCollapse);
    D.state = end_state;
    D.n_outer += 1;
    if (k + 1 > D.ksub_max) D.ksub_max = (int32_t)(k + 1);
}

// after the force pass of substep k, for systems whose continuity pass does
// not end the substep itself (one block per system)
__global__ __launch_bounds__(kBlock) void k_dt_substep(DevArrays A, int64_t group, int G)
{
    const int s = blockIdx.x;
    SysDyn& D = A.sd[s];
    const SysConst& S = A.sc[s];
    if (S.fuse_dt) return;
    const int st = D.state;
    if (st == kEnding) {
        if (threadIdx.x == 0) D.state = kEnded;
        return;
    }
    if (st != kSubstepping) return;  // block-uniform
    double vmax[2];
    reduce_vmax<16>(A, S, kBlock / G, vmax);
    if (threadIdx.x != 0) return;
    if (A.work) atomicOr(A.work + group, 1);
    const long long k = D.ksub;
    const double dt = D.dt[k & 1];
    commit_substep(D, k, dt, vmax, end_substep(S, D.dt_ad, D.tau, dt, D.health, vmax), kEnding);
}

__global__ void k_reset_ksub_max(DevArrays A)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < A.nsys) A.sd[s].ksub_max = 0;
}

// ---------------------------------------------------------------------------
// substep pair pass 1: colour gradient (Eq. 22) of interface particles
// ---------------------------------------------------------------------------

// The substep as it starts, for the continuity pass that ends it: taken by
// the first thread of the system's first block (no pass before the
// continuity pass reads these fields; taking it twice stores the same values)
template <int G>
__device__ __forceinline__ void colour_snapshot(const DevArrays& A, const Slot& c, SysDyn& Dy)
{
    if (A.mode == 0 && threadIdx.x == 0 && logical_block() * (kBlock / G) == A.sc[c.s].p_off) {
        Dy.sub_state = Dy.state;
        Dy.sub_health = Dy.health;
        Dy.sub_ksub = Dy.ksub;
        Dy.sub_tau = Dy.tau;
    }
}

template <typename R, int D, bool PK = false>
__global__ __launch_bounds__(kBlock) void k_colour(DevArrays A)
{
    constexpr int G = Lanes<D>::G;
    int g;
    const int64_t i = group_slot<G>(g);
    if (i >= A.P) return;
    if (A.state_first) {
        const Slot c0 = lookup_slot(A, i);
        if (c0.s < 0) return;
        colour_snapshot<G>(A, c0, A.sd[c0.s]);
        if (!substep_on(A.sd[c0.s], A.mode)) return;
        // a wave without interface particles (most of a large pool's) exits
        // before any other load
        if (!__any(c0.lane && (A.flags[i] & kFlagInterface))) return;
    }
    // loads that need only the slot, issued together
    using GT = typename GeoT<R, D>::T;
    const GT* geo = (const GT*)A.geo;
    NbrList<G, PassChunk<R, D, Pass::Colour>::N> nl;
    nl.start(A, i, g);
    const int fl = A.flags[i];
    const int cnt_i = A.ncount[i];
    const GT gi_i = geo[i];
    const Slot c = lookup_slot(A, i);
    if (c.s < 0) return;
    SysDyn& Dy = A.sd[c.s];
    colour_snapshot<G>(A, c, Dy);
    if (!substep_on(Dy, A.mode)) return;
    const bool on = c.lane && (fl & kFlagInterface);
    if (!__any(on)) return;  // wave without interface particles
    const SysConst& S = A.sc[c.s];
    // the substep's volumes: packed, from the {v, p} records
    const int slot = A.mode ? 0 : (int)(Dy.ksub & 1);
    const Q4<R>* th = (const Q4<R>*)(PK ? A.vbuf[0] : A.th[slot]);
    const FromPressure<R> fp(S);
    R cellr[3] = {(R)S.cell[0], (R)S.cell[1], (R)S.cell[2]};
    const R inv_h = (R)S.inv_h, coef = (R)S.dw_coef;
    const GT gi = on ? gi_i : GT{};
    const int cnt = on ? cnt_i : 0;
    const int phi = Geo<R>::phase(gi);
    R gsum[3] = {0, 0, 0};
    nl.run(
        g, cnt, [&](uint32_t j) { return GRecs<GT, R, 1>{geo[j], {th[j]}}; },
        [&](uint32_t ent, const GRecs<GT, R, 1>& rj) {
            const GT gj = rj.g;
            const int phj = Geo<R>::phase(gj);
            if (phj == phi || phj == kWall) return;  // walls carry no colour
            R r[3];
            Geo<R>::template rij<D>(gi, gj, ent, S, cellr, r);
            const R r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const R inv_r = rsqrt_dist<R>(r2);
            const R Vj = PK ? fp.m(phj) * recip<R>(fp.rho(phj, rj.q[0].w)) : rj.q[0].y;
            const R f = wendland_dw<R>(r2 * inv_r * inv_h, coef) * Vj * inv_r;
            gsum[0] += f * r[0];
            gsum[1] += f * r[1];
            if (D == 3) gsum[2] += f * r[2];
        });
    for (int a = 0; a < D; ++a) gsum[a] = group_sum<G>(gsum[a]);
    if (!on || g != 0) return;
    // 2 phi_i = 2 rho0_i / (rho0_i + rho0_j) for a neighbour of the other fluid
    const R two_phi = (R)(2.0 * S.rho0[phi] / (S.rho0[0] + S.rho0[1]));
    for (int a = 0; a < D; ++a) gsum[a] *= two_phi;
    const R gg = gsum[0] * gsum[0] + gsum[1] * gsum[1] + gsum[2] * gsum[2];
    const R invg = gg > R(0) ? rsqrt_r<R>(gg) : R(0);
    ((Q4<R>*)A.col)[i] = Q4<R>{gsum[0], gsum[1], gsum[2], invg};
    if (A.mode == 1)
        for (int a = 0; a < 3; ++a) A.r_gradc[3 * i + a] = a < D ? (double)gsum[a] : 0.0;
}

// ---------------------------------------------------------------------------
// substep pair pass 2: Riemann pressure (Eqs. 7-12), surface stress divergence
// with the projected penalty (Eqs. 24, 27, 30, 33), kick
// ---------------------------------------------------------------------------

template <typename R, int D, bool PK = false, bool WL = true>
__global__ __launch_bounds__(kBlock) void k_force(DevArrays A)
{
    constexpr int G = Lanes<D>::G;
    int g;
    const int64_t i = group_slot<G>(g);
    if (i >= A.P) return;
    if (A.state_first) {
        const Slot c0 = lookup_slot(A, i);
        if (c0.s < 0 || !substep_on(A.sd[c0.s], A.mode)) return;
    }
    // loads that need only the slot, issued together
    using GT = typename GeoT<R, D>::T;
    const GT* geo = (const GT*)A.geo;
    const Q4<R>* col = (const Q4<R>*)A.col;
    NbrList<G, PassChunk<R, D, Pass::Force>::N> nl;
    nl.start(A, i, g);
    const int fl = A.flags[i];
    const int cnt_i = A.ncount[i];
    const GT gi_i = geo[i];
    // particles away from the interface all read entry 0 (one cache line)
    const Q4<R> ci_i = col[(fl & kFlagNearInterface) ? i : 0];
    const Q4<R> av_i = ((const Q4<R>*)A.av)[i];
    double vel_i[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) vel_i[a] = A.vel[a][i];
    const Slot c = lookup_slot(A, i);
    if (c.s < 0) return;
    SysDyn& Dy = A.sd[c.s];
    if (!substep_on(Dy, A.mode)) return;  // wave-uniform
    const SysConst& S = A.sc[c.s];
    const int64_t kk = A.mode ? 0 : Dy.ksub;
    const int slot = (int)(kk & 1);
    // packed: the {v, p} records as the substep starts, and the kicked ones
    const Q4<R>* th = (const Q4<R>*)A.th[slot];
    const Q4<R>* vin = (const Q4<R>*)A.vbuf[PK ? 0 : slot];
    Q4<R>* vout = (Q4<R>*)A.vbuf[PK ? 1 : slot ^ 1];
    const FromPressure<R> fpr(S);
    R cellr[3] = {(R)S.cell[0], (R)S.cell[1], (R)S.cell[2]};
    const R c0 = (R)S.c0, three_inv_c0 = (R)(3.0 * S.inv_c0);
    // the kernel gradient's constants: 1 / (2h) and coef / h (W' below)
    const R half_inv_h = (R)(0.5 * S.inv_h), coef_h = (R)(S.dw_coef * S.inv_h);
    const GT gi = c.lane ? gi_i : GT{};
    const int phi = Geo<R>::phase(gi);
    Q4<R> ti{1, 0, 0, 0}, vi{0, 0, 0, 0};
    if (c.lane) {
        vi = vin[i];
        ti = PK ? fpr(phi, vi.w) : th[i];
    }
    const R m_i = PK ? fpr.m(phi) : R(0);  // packed: the fluid's particle mass
    const R c0_rho_i = c0 * ti.x;
    const bool wall_i = phi == kWall;  // a wall particle has no rates and never moves
    const int cnt = (c.lane && !wall_i) ? cnt_i : 0;
    const bool surface = c.lane && !wall_i && (fl & kFlagNearInterface) && !(S.flags & kNoSurface);
    const Q4<R> ci = surface ? ci_i : Q4<R>{0, 0, 0, 0};
    const bool penalty = !(S.flags & kNoPenalty);
    // cross pairs: the neighbour's gradient enters negated (one colour field,
    // Eq. 25) unless the printed own-phase average is asked for
    const bool single = (S.flags & kGbarOwnPhaseAverage) == 0;
    const bool r3 = (S.flags & kPenaltyR3) != 0;
    const R gamma = (R)S.gamma;
    const R xg = (R)(S.xi * S.gamma);
    const R rho0_i = (R)S.rho0[phi & 1], rho0_o = (R)S.rho0[(phi & 1) ^ 1];
    const R grav[3] = {(R)S.grav[0], (R)S.grav[1], (R)S.grav[2]};
    const R phi_i_x = rho0_i / (rho0_i + rho0_o);  // phi_i for a cross pair
    const R phi_j_x = rho0_o / (rho0_i + rho0_o);
    const R pen_x = R(-4) * phi_i_x * phi_j_x * xg;
    const R gni = (ci.x * ci.x + ci.y * ci.y + ci.z * ci.z) * ci.w;  // |grad C_i|
    R sp[3] = {0, 0, 0}, ss[3] = {0, 0, 0};
    constexpr int NR = PK ? 2 : 3;
    nl.run(
        g, cnt,
        [&](uint32_t j) {
            if constexpr (PK) return GRecs<GT, R, 1>{geo[j], {vin[j]}};
            else return GRecs<GT, R, 2>{geo[j], {th[j], vin[j]}};
        },
        [&](uint32_t ent, const GRecs<GT, R, NR - 1>& rj) {
            const GT gj = rj.g;
            R r[3];
            Geo<R>::template rij<D>(gi, gj, ent, S, cellr, r);
            const R r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const R inv_r = rsqrt_dist<R>(r2);
            const R rr = r2 * inv_r;
            // W'(r) = coef (r/h) (1 - r/(2h))^3
            const R a = R(1) - rr * half_inv_h;
            const R dW = coef_h * rr * (a * a * a);
            const Q4<R> vj = rj.q[NR - 2];
            const int phj = Geo<R>::phase(gj);
            // packed: rho_j from the pressure, V_j = m_j / rho_j folded into the
            // one reciprocal below
            R rhoR, pR, mR = m_i, Vj = 0;
            if constexpr (PK) {
                rhoR = fpr.rho(phj, vj.w);
                pR = vj.w;
                mR = fpr.m(phj);
            } else {
                rhoR = rj.q[0].x;
                pR = rj.q[0].z;
                Vj = rj.q[0].y;
            }
            // Eq. 10 states (U = -v . e), Eq. 11 limiter, Eqs. 8 and 12:
            // U_L - U_R = (v_j - v_i) . e
            R dU;
            const bool wall_j = WL && phj == kWall;  // WL: the pool holds walls
            if (wall_j) {
                // the wall's mirrored state: rho_R = rho_i, U_R = 2 U_w - U_L,
                // p_R = p_i - rho_i g . r_ij, volume V_i
                const R UL = -(vi.x * r[0] + vi.y * r[1] + vi.z * r[2]) * inv_r;
                const R Uw = -(vj.x * r[0] + vj.y * r[1] + vj.z * r[2]) * inv_r;
                dU = UL - (R(2) * Uw - UL);
                rhoR = ti.x;
                pR = ti.z - ti.x * (grav[0] * r[0] + grav[1] * r[1] + grav[2] * r[2]);
                mR = m_i;
                Vj = ti.y;
            } else {
                dU = ((vj.x - vi.x) * r[0] + (vj.y - vi.y) * r[1] + (vj.z - vi.z) * r[2]) * inv_r;
            }
            // beta = min(3 max(dU / c0, 0), 1)
            const R beta = fmin(fmax(dU * three_inv_c0, R(0)), R(1));
            const R num = ti.x * pR + rhoR * ti.z + (beta * c0_rho_i) * rhoR * dU;
            // P* V_j = num V_j / (rho_i + rho_R), summed as P* V_j W' r_ij / r
            R fp;
            R qv = 0;  // packed: V_j / (m_j (rho_i + rho_R))
            if constexpr (PK) {
                qv = recip<R>((ti.x + rhoR) * rhoR);
                fp = num * mR * qv * dW;
            } else {
                fp = num * recip<R>(ti.x + rhoR) * dW * Vj;
            }
            const R fpr_ = fp * inv_r;
            sp[0] += fpr_ * r[0];
            sp[1] += fpr_ * r[1];
            if (D == 3) sp[2] += fpr_ * r[2];
            if (!surface || wall_j) return;  // walls carry no colour
            if constexpr (PK) Vj = mR * (ti.x + rhoR) * qv;
            const R e[3] = {r[0] * inv_r, r[1] * inv_r, r[2] * inv_r};
            const bool same = Geo<R>::phase(gj) == phi;
            const Q4<R> cj = col[ent & kNbrIndexMask];
            const R gnj = (cj.x * cj.x + cj.y * cj.y + cj.z * cj.z) * cj.w;
            // Pi e = gamma (|g| e - g (g . e) / |g|)
            const R gie = (ci.x * e[0] + ci.y * e[1] + ci.z * e[2]) * ci.w;
            const R gje = (cj.x * e[0] + cj.y * e[1] + cj.z * e[2]) * cj.w;
            const R wi = same ? R(1) : R(2) * phi_j_x;
            const R wj = same ? R(1) : R(2) * phi_i_x;
            R se[3];
            se[0] = gamma * (wi * (gni * e[0] - ci.x * gie) + wj * (gnj * e[0] - cj.x * gje));
            se[1] = gamma * (wi * (gni * e[1] - ci.y * gie) + wj * (gnj * e[1] - cj.y * gje));
            se[2] = gamma * (wi * (gni * e[2] - ci.z * gie) + wj * (gnj * e[2] - cj.z * gje));
            const R fs = dW * Vj;
            ss[0] += fs * se[0];
            ss[1] += fs * se[1];
            if (D == 3) ss[2] += fs * se[2];
            if (!penalty) return;
            // Eq. 27 and Eq. 30 (reading R1): Chat grad W = dW [C e - (gbar.r) gbar/|gbar|]
            const R sgn = (single && !same) ? R(-1) : R(1);
            const R gb[3] = {R(0.5) * (ci.x + sgn * cj.x), R(0.5) * (ci.y + sgn * cj.y),
                             R(0.5) * (ci.z + sgn * cj.z)};
            const R gb2 = gb[0] * gb[0] + gb[1] * gb[1] + gb[2] * gb[2];
            const R gbr = gb[0] * r[0] + gb[1] * r[1] + gb[2] * r[2];
            const R inv_gb = gb2 > R(0) ? rsqrt_r<R>(gb2) : R(0);
            const R C = same ? R(0) : R(1);
            R q[3];
            if (r3) {
                const R sc = dW * (C - gbr * gbr * inv_gb * inv_r);
                q[0] = sc * e[0];
                q[1] = sc * e[1];
                q[2] = sc * e[2];
            } else {
                const R t = gbr * inv_gb;
                q[0] = dW * (C * e[0] - t * gb[0]);
                q[1] = dW * (C * e[1] - t * gb[1]);
                q[2] = dW * (C * e[2] - t * gb[2]);
            }
            // Nbar q = (n_i (n_i . q) + n_j (n_j . q)) / 2 with n = g / |g|
            const R niq = (ci.x * q[0] + ci.y * q[1] + ci.z * q[2]) * ci.w * ci.w;
            const R njq = (cj.x * q[0] + cj.y * q[1] + cj.z * q[2]) * cj.w * cj.w;
            R Nq[3];
            Nq[0] = R(0.5) * (ci.x * niq + cj.x * njq);
            Nq[1] = R(0.5) * (ci.y * niq + cj.y * njq);
            Nq[2] = R(0.5) * (ci.z * niq + cj.z * njq);
            const R pc = (same ? xg : pen_x) * inv_r * Vj;
            if (same) {
                // Tbar q = q - Nbar q
                ss[0] += pc * (q[0] - Nq[0]);
                ss[1] += pc * (q[1] - Nq[1]);
                if (D == 3) ss[2] += pc * (q[2] - Nq[2]);
            } else {
                ss[0] += pc * Nq[0];
                ss[1] += pc * Nq[1];
                if (D == 3) ss[2] += pc * Nq[2];
            }
        });
    for (int a = 0; a < D; ++a) {
        sp[a] = group_sum<G>(sp[a]);
        ss[a] = group_sum<G>(ss[a]);
    }
    unsigned long long m0 = 0, m1 = 0;
    if (c.lane && g == 0 && wall_i) {
        // a wall keeps its velocity: the record of the kicked velocities
        // carries it on; it has no rates
        vout[i] = vi;
        if (A.mode == 1)
            for (int a = 0; a < 3; ++a) A.r_acc[3 * i + a] = A.r_accp[3 * i + a] = A.r_accs[3 * i + a] = 0.0;
    } else if (c.lane && g == 0) {
        const R inv_rho = R(1) / ti.x;
        const R avv[3] = {av_i.x, av_i.y, av_i.z};
        double acc[3];
        for (int a = 0; a < 3; ++a)
            acc[a] = a < D ? (double)(R(-2) * inv_rho * sp[a]) + (double)(inv_rho * ss[a]) +
                                 (double)avv[a] + S.grav[a]
                           : 0.0;
        if (A.mode == 1) {
            for (int a = 0; a < 3; ++a) {
                A.r_acc[3 * i + a] = acc[a];
                A.r_accp[3 * i + a] = a < D ? (double)(R(-2) * inv_rho * sp[a]) : 0.0;
                A.r_accs[3 * i + a] = a < D ? (double)(inv_rho * ss[a]) : 0.0;
            }
            vout[i] = vi;
        } else {
            const double dt = Dy.dt[kk & 1];
            double v[3] = {0.0, 0.0, 0.0};
            double v2 = 0.0;
            bool bad = false;
            for (int a = 0; a < D; ++a) {
                v[a] = vel_i[a] + dt * acc[a];
                A.vel[a][i] = v[a];
                v2 += v[a] * v[a];
                bad |= !isfinite(v[a]);
            }
            if (bad) flag_health(Dy, kHealthNonFinite);
            // packed: the pressure rides on to the continuity pass
            vout[i] = Q4<R>{(R)v[0], (R)v[1], (R)v[2], PK ? vi.w : (R)0};
            unsigned long long bits = (unsigned long long)__double_as_longlong(sqrt(v2));
            if (phi == 0) m0 = bits;
            else m1 = bits;  // (a wall never gets here)
        }
    }
    if (A.mode == 1) return;  // block-uniform
    // block maximum: one partial per block (a block lies in one system)
    __shared__ unsigned long long red[2 * (kBlock / kWave)];
    m0 = wave_max_u64(m0);
    m1 = wave_max_u64(m1);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[2 * wv] = m0;
        red[2 * wv + 1] = m1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / kWave; ++k) {
            m0 = red[2 * k] > m0 ? red[2 * k] : m0;
            m1 = red[2 * k + 1] > m1 ? red[2 * k + 1] : m1;
        }
        const int64_t lb = logical_block();
        A.vpart[2 * lb] = m0;
        A.vpart[2 * lb + 1] = m1;
    }
}

// ---------------------------------------------------------------------------
// substep pair pass 3: continuity with the new velocity (Eq. 6 with Eq. 9),
// second half-step, and the first half-step of the next substep
// ---------------------------------------------------------------------------

template <typename R, int D, bool PK = false, bool WL = true>
__global__ __launch_bounds__(kBlock) void k_continuity(DevArrays A, int64_t group)
{
    constexpr int G = Lanes<D>::G;
    int g;
    const int64_t i = group_slot<G>(g);
    if (i >= A.P) return;
    if (A.state_first) {
        // the same exits as below, before any slot load
        const Slot c0 = lookup_slot(A, i);
        if (c0.s < 0) return;
        const SysDyn& D0 = A.sd[c0.s];
        const bool idle = A.mode == 1           ? !D0.stepping
                          : A.sc[c0.s].fuse_dt ? D0.sub_state != kSubstepping
                                               : D0.state != kSubstepping && D0.state != kEnding;
        if (idle) return;
    }
    // loads that need only the slot, issued together
    using GT = typename GeoT<R, D>::T;
    const GT* geo = (const GT*)A.geo;
    NbrList<G, PassChunk<R, D, Pass::Continuity>::N> nl;
    nl.start(A, i, g);
    const int cnt_i = A.ncount[i];
    const GT gi_i = geo[i];
    // FP64 state of the particle for the update that follows the sum
    const double rho_i = A.rho[i], mass_i = A.mass[i];
    double pos_i[3] = {0.0, 0.0, 0.0}, vel_i[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) {
        pos_i[a] = A.pos[a][i];
        vel_i[a] = A.vel[a][i];
    }
    const Slot c = lookup_slot(A, i);
    if (c.s < 0) return;
    SysDyn& Dy = A.sd[c.s];
    const SysConst& S = A.sc[c.s];
    // the substep this pass completes
    int64_t kk = 0;
    int st = kSubstepping;
    const bool fused = A.mode == 0 && S.fuse_dt;
    unsigned long long vbits[2] = {0ull, 0ull};
    // a fused system's partials: at most 4 per thread, which 2D loads before
    // the pair sum and folds after it (3D reduces them at once: its pair sum
    // has no registers to spare)
    static_assert(kFuseDtEntries <= 4 * kBlock, "partials of a fused system");
    VParts<4> vp;
    if (A.mode == 1) {
        if (!Dy.stepping) return;
    } else if (fused) {
        // This pass ends the substep: every block reduces the system's |v|
        // maxima of the force pass and decides from the substep as it started
        // (after the pair sum below), so all blocks decide alike.
        if (Dy.sub_state != kSubstepping) return;  // block-uniform
        kk = Dy.sub_ksub;
        if constexpr (D == 2) {
            int64_t e0, e1;
            vmax_range(S, kBlock / G, e0, e1);
            vmax_load<4>(A, e0 + threadIdx.x, e1, vp);
        } else {
            reduce_vmax_bits<4>(A, S, kBlock / G, vbits);
        }
    } else {
        // the substep pass has ended the substep (and advanced ksub)
        st = Dy.state;
        if (st != kSubstepping && st != kEnding) return;
        kk = Dy.ksub - 1;
    }
    const int slot = (int)(kk & 1);
    // packed: the kicked {v, p} records
    const Q4<R>* th = (const Q4<R>*)A.th[slot];
    const Q4<R>* vk = (const Q4<R>*)A.vbuf[PK ? 1 : slot ^ 1];
    const FromPressure<R> fpr(S);
    R cellr[3] = {(R)S.cell[0], (R)S.cell[1], (R)S.cell[2]};
    const R inv_h = (R)S.inv_h, coef = (R)S.dw_coef;
    const R inv_c0 = (R)S.inv_c0;
    const GT gi = c.lane ? gi_i : GT{};
    Q4<R> ti{1, 0, 0, 0}, vi{0, 0, 0, 0};
    if (c.lane) {
        vi = vk[i];
        ti = PK ? fpr(Geo<R>::phase(gi), vi.w) : th[i];
    }
    const bool wall_i = Geo<R>::phase(gi) == kWall;  // a wall keeps its density
    const int cnt = (c.lane && !wall_i) ? cnt_i : 0;
    const R grav[3] = {(R)S.grav[0], (R)S.grav[1], (R)S.grav[2]};
    R s = 0;
    constexpr int NR = PK ? 2 : 3;
    nl.run(
        g, cnt,
        [&](uint32_t j) {
            if constexpr (PK) return GRecs<GT, R, 1>{geo[j], {vk[j]}};
            else return GRecs<GT, R, 2>{geo[j], {th[j], vk[j]}};
        },
        [&](uint32_t ent, const GRecs<GT, R, NR - 1>& rj) {
            const GT gj = rj.g;
            R r[3];
            Geo<R>::template rij<D>(gi, gj, ent, S, cellr, r);
            const R r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const R inv_r = rsqrt_dist<R>(r2);
            const R dW = wendland_dw<R>(r2 * inv_r * inv_h, coef);
            const Q4<R> vj = rj.q[NR - 2];
            const int phj = Geo<R>::phase(gj);
            const R vie = (vi.x * r[0] + vi.y * r[1] + vi.z * r[2]) * inv_r;
            const R vje = (vj.x * r[0] + vj.y * r[1] + vj.z * r[2]) * inv_r;
            // U* = (rho_i U_L + rho_j U_R + (p_i - p_j)/c0) / (rho_i + rho_j), U = -v.e,
            // so v_i.e + U* = (rho_j (v_i - v_j).e + (p_i - p_j)/c0) / (rho_i + rho_j);
            // against a wall's mirror (rho_R = rho_i, U_R = 2 U_w - U_L,
            // p_R = p_i - rho_i g . r_ij, volume V_i): U* = U_w + g . r_ij / (2 c0)
            if (WL && phj == kWall) {  // WL: the pool holds walls
                const R Ustar = -vje + (grav[0] * r[0] + grav[1] * r[1] + grav[2] * r[2]) * R(0.5) * inv_c0;
                s += (vie + Ustar) * dW * ti.y;
                return;
            }
            R rhoj, pj, q;
            if constexpr (PK) {  // V_j / (rho_i + rho_j) = m_j / ((rho_i + rho_j) rho_j)
                rhoj = fpr.rho(phj, vj.w);
                pj = vj.w;
                q = fpr.m(phj) * recip<R>((ti.x + rhoj) * rhoj);
            } else {
                rhoj = rj.q[0].x;
                pj = rj.q[0].z;
                q = rj.q[0].y * recip<R>(ti.x + rhoj);
            }
            s += (rhoj * (vie - vje) + (ti.z - pj) * inv_c0) * q * dW;
        });
    s = group_sum<G>(s);
    // the acoustic steps of this substep and, if another one follows in the
    // advection step, of the next
    const double dt = Dy.dt[kk & 1];
    double dt2 = 0.0;
    bool next = st == kSubstepping;
    if (fused) {
        if constexpr (D == 2) {
            unsigned long long m0 = 0, m1 = 0;
            vmax_fold<4>(vp, m0, m1);
            vmax_block(m0, m1, vbits);
        }
        const double vmax[2] = {__longlong_as_double((long long)vbits[0]),
                                __longlong_as_double((long long)vbits[1])};
        const SubstepEnd e = end_substep(S, Dy.dt_ad, Dy.sub_tau, dt, Dy.sub_health, vmax);
        next = e.next;
        dt2 = e.dt_next;
        // the system's first block stores the decision (no block of this
        // pass reads the fields it changes)
        if (threadIdx.x == 0 && logical_block() * (kBlock / G) == S.p_off) {
            if (A.work) atomicOr(A.work + group, 1);
            commit_substep(Dy, kk, dt, vmax, e, kEnded);
        }
    } else if (next) {
        dt2 = Dy.dt[(kk + 1) & 1];
    }
    if (!c.lane || g != 0) return;
    const double drho = wall_i ? 0.0 : 2.0 * (double)ti.x * (double)s;
    if (A.mode == 1) {
        A.r_drho[i] = drho;
        return;
    }
    if (wall_i) {
        if (next) {
            if (PK) ((Q4<R>*)A.vbuf[0])[i] = vi;
            else ((Q4<R>*)A.th[slot ^ 1])[i] = ti;
        }
        return;
    }
    double rho = rho_i + 0.5 * dt * drho;
    for (int a = 0; a < D; ++a) pos_i[a] += 0.5 * dt * vel_i[a];
    if (next) {
        rho += 0.5 * dt2 * drho;
        for (int a = 0; a < D; ++a) pos_i[a] += 0.5 * dt2 * vel_i[a];
        const int ph = Geo<R>::phase(gi);
        const R p = (R)(S.c0sq * (rho - S.rho0[ph]));
        if (PK) ((Q4<R>*)A.vbuf[0])[i] = Q4<R>{vi.x, vi.y, vi.z, p};
        else ((Q4<R>*)A.th[slot ^ 1])[i] = Q4<R>{(R)rho, (R)(mass_i / rho), p, (R)0};
    }
    for (int a = 0; a < D; ++a) A.pos[a][i] = pos_i[a];
    A.rho[i] = rho;
    A.drho[i] = drho;
    if (!(rho > 0.0)) flag_health(Dy, isfinite(rho) ? kHealthDensity : kHealthNonFinite);
}

// ---------------------------------------------------------------------------
// observables: per-wave partial sums in a fixed butterfly order, then one
// block per system summing its waves in a fixed strided order and a fixed tree
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_maxd(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// pass 0: momentum(3) kinetic mass(2) volume(2) vmax(2) m x of fluid k(3)
// pass 1: moment2 about the centroid (6) p_in n_in p_out n_out
template <int D>
__global__ __launch_bounds__(kWave) void k_obs_partial(DevArrays A, int pass)
{
    const int64_t w = blockIdx.x;
    const int64_t i = w * kWave + threadIdx.x;
    if (i >= A.P) return;
    int s = system_of_wave(A, w);
    s = __builtin_amdgcn_readfirstlane(s);
    if (s < 0) return;
    const SysConst& S = A.sc[s];
    // observables are of the fluids: wall particles are left out
    const bool lane = i < S.p_off + S.p_n && A.phase[i] != kWall;
    double f[kObsPart];
    for (int k = 0; k < kObsPart; ++k) f[k] = 0.0;
    if (lane) {
        const double m = A.mass[i];
        const int ph = A.phase[i];
        double x[3] = {0, 0, 0}, v[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            x[a] = A.pos[a][i];
            v[a] = A.vel[a][i];
        }
        if (pass == 0) {
            double v2 = 0.0;
            for (int a = 0; a < D; ++a) {
                f[a] = m * v[a];
                v2 += v[a] * v[a];
            }
            f[3] = 0.5 * m * v2;
            f[4 + ph] = m;
            f[6 + ph] = m / A.rho[i];
            f[8 + ph] = sqrt(v2);
            if (ph == 0)
                for (int a = 0; a < D; ++a) f[10 + a] = m * x[a];
        } else {
            const double* o = A.obs_out + (int64_t)s * kObsOut;
            double dx[3] = {0, 0, 0};
            double r2 = 0.0;
            for (int a = 0; a < D; ++a) {
                dx[a] = x[a] - o[10 + a];
                r2 += dx[a] * dx[a];
            }
            if (ph == 0) {
                f[0] = m * dx[0] * dx[0];
                f[1] = m * dx[0] * dx[1];
                f[2] = m * dx[0] * dx[2];
                f[3] = m * dx[1] * dx[1];
                f[4] = m * dx[1] * dx[2];
                f[5] = m * dx[2] * dx[2];
            }
            const double r = sqrt(r2);
            const double p = S.c0sq * (A.rho[i] - S.rho0[ph]);
            const double req = o[13];
            if (ph == 0 && r < req - 3.0 * S.h) {
                f[6] = p;
                f[7] = 1.0;
            }
            if (ph == 1 && r > req + 3.0 * S.h) {
                f[8] = p;
                f[9] = 1.0;
            }
        }
    }
    for (int k = 0; k < kObsPart; ++k) {
        const bool is_max = pass == 0 && (k == 8 || k == 9);
        f[k] = is_max ? wave_maxd(f[k]) : wave_sum(f[k]);
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < kObsPart; ++k) A.obs_part[w * kObsPart + k] = f[k];
}

__global__ __launch_bounds__(kBlock) void k_obs_final(DevArrays A, int pass)
{
    __shared__ double lds[kBlock];
    const int s = blockIdx.x;
    const SysConst& S = A.sc[s];
    const int64_t w0 = S.p_off / kWave, w1 = (S.p_off + S.p_n + kWave - 1) / kWave;
    double* o = A.obs_out + (int64_t)s * kObsOut;
    // thread t accumulates waves t, t + 256, ... in that order, every quantity
    // at once: the 128-byte records of U waves are in flight together
    constexpr int U = 2;
    static_assert(kObsPart % 2 == 0, "16-byte loads");
    double acc[kObsPart];
    for (int k = 0; k < kObsPart; ++k) acc[k] = 0.0;
    for (int64_t w = w0 + threadIdx.x; w < w1; w += U * kBlock) {
        double2 r[U][kObsPart / 2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t wu = w + (int64_t)u * kBlock;
            const double2* src = (const double2*)(A.obs_part + (wu < w1 ? wu : w) * kObsPart);
#pragma unroll
            for (int k = 0; k < kObsPart / 2; ++k) r[u][k] = src[k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (w + (int64_t)u * kBlock >= w1) break;
#pragma unroll
            for (int k = 0; k < kObsPart; ++k) {
                const double v = (k & 1) ? r[u][k >> 1].y : r[u][k >> 1].x;
                const bool is_max = pass == 0 && (k == 8 || k == 9);
                acc[k] = is_max ? fmax(acc[k], v) : acc[k] + v;
            }
        }
    }
    for (int k = 0; k < kObsPart; ++k) {
        const bool is_max = pass == 0 && (k == 8 || k == 9);
        lds[threadIdx.x] = acc[k];
        __syncthreads();
        for (int h = kBlock / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h)
                lds[threadIdx.x] = is_max ? fmax(lds[threadIdx.x], lds[threadIdx.x + h])
                                          : lds[threadIdx.x] + lds[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) o[(pass == 0 ? 0 : 16) + k] = lds[0];
        __syncthreads();
    }
    if (pass == 0 && threadIdx.x == 0) {
        // centroid of fluid k and equivalent radius of its volume
        const double mk = o[4];
        for (int a = 0; a < 3; ++a) o[10 + a] = mk > 0.0 ? o[10 + a] / mk : 0.0;
        const double vol = o[6];
        o[13] = S.dim == 2 ? sqrt(vol / M_PI) : cbrt(3.0 * vol / (4.0 * M_PI));
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline dim3 slot_grid(int64_t P, int lanes = 1)
{
    int64_t nb = (P * lanes + kBlock - 1) / kBlock;
    nb = (nb + 7) / 8 * 8;
    return dim3((unsigned)nb);
}

static inline dim3 flat_grid(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }
static inline dim3 sys_grid(int n) { return dim3((unsigned)((n + 63) / 64)); }

template <typename K, typename... Args>
static void go(K kernel, dim3 grid, dim3 block, hipStream_t st, Ev ev, Args... args)
{
    if (ev.start || ev.stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ev.start, ev.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

__global__ void k_empty() {}

void launch_empty(const Launch& L, Ev ev) { go(k_empty, dim3(1), dim3(kWave), L.stream, ev); }

void launch_fill_i32(const Launch& L, int32_t* p, int64_t n, int32_t v)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, flat_grid(n), dim3(kBlock), 0, L.stream, p, n, v);
}

void launch_set_stepping(const Launch& L, const DevArrays& A, const int32_t* mask)
{
    hipLaunchKernelGGL(k_set_stepping, sys_grid(A.nsys), dim3(64), 0, L.stream, A, mask);
}

void launch_reset_ksub_max(const Launch& L, const DevArrays& A)
{
    hipLaunchKernelGGL(k_reset_ksub_max, sys_grid(A.nsys), dim3(64), 0, L.stream, A);
}

void launch_set_targets(const Launch& L, const DevArrays& A, const long long* targets)
{
    hipLaunchKernelGGL(k_set_targets, sys_grid(A.nsys), dim3(64), 0, L.stream, A, targets);
}

void launch_bin(const Launch& L, const DevArrays& A, int64_t group)
{
    // the cell counts are zero on entry: cleared when the arrays are
    // allocated and by every binning after the scan has consumed them
    const int64_t ncells = A.C;
    if (L.dim == 2)
        hipLaunchKernelGGL(k_key<2>, slot_grid(A.P), dim3(kBlock), 0, L.stream, A, group);
    else
        hipLaunchKernelGGL(k_key<3>, slot_grid(A.P), dim3(kBlock), 0, L.stream, A, group);
    const bool small = ncells <= kScanSmall;
    if (small) {
        hipLaunchKernelGGL(k_scatter_small, slot_grid(A.P), dim3(kBlock), 0, L.stream, A, ncells);
    } else {
        const int64_t ntiles = (ncells + kScanTile - 1) / kScanTile;
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)ntiles), dim3(kBlock), 0, L.stream, A.cell_cnt,
                           ncells, A.scan_part);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, L.stream, A.scan_part, ntiles);
        hipLaunchKernelGGL(k_scan_final, dim3((unsigned)ntiles), dim3(kBlock), 0, L.stream, A.cell_cnt,
                           ncells, A.scan_part, A.cell_start);
        hipLaunchKernelGGL(k_scatter, slot_grid(A.P), dim3(kBlock), 0, L.stream, A);
    }
    const int64_t clear_n = small ? ncells : 0;
    if (L.dim == 2)
        hipLaunchKernelGGL(k_rank<2>, slot_grid(A.P), dim3(kBlock), 0, L.stream, A, clear_n);
    else
        hipLaunchKernelGGL(k_rank<3>, slot_grid(A.P), dim3(kBlock), 0, L.stream, A, clear_n);
}

#define RSPH_DISPATCH(KERNEL, LANES2, LANES3, EV, ...)                                                 \
    do {                                                                                           \
        if (L.fp64) {                                                                              \
            if (L.dim == 2)                                                                        \
                go(KERNEL<double, 2>, slot_grid(A.P, LANES2), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
            else                                                                                   \
                go(KERNEL<double, 3>, slot_grid(A.P, LANES3), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
        } else {                                                                                   \
            if (L.dim == 2)                                                                        \
                go(KERNEL<float, 2>, slot_grid(A.P, LANES2), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
            else                                                                                   \
                go(KERNEL<float, 3>, slot_grid(A.P, LANES3), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
        }                                                                                          \
    } while (0)

constexpr int G2 = Lanes<2>::G;
constexpr int G3 = Lanes<3>::G;

// the substep passes: the packed form when every fluid's masses are uniform,
// and without the wall branches when no system holds walls (PK and WL are
// the template arguments after the record type and dimension)
#define RSPH_GO_PW(KERNEL, PKV, WLV, EV, ...)                                                      \
    do {                                                                                           \
        if (L.fp64) {                                                                              \
            if (L.dim == 2)                                                                        \
                go(KERNEL<double, 2, PKV, WLV>, slot_grid(A.P, G2), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
            else                                                                                   \
                go(KERNEL<double, 3, PKV, WLV>, slot_grid(A.P, G3), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
        } else {                                                                                   \
            if (L.dim == 2)                                                                        \
                go(KERNEL<float, 2, PKV, WLV>, slot_grid(A.P, G2), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
            else                                                                                   \
                go(KERNEL<float, 3, PKV, WLV>, slot_grid(A.P, G3), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
        }                                                                                          \
    } while (0)
#define RSPH_DISPATCH_PW(KERNEL, EV, ...)                                                          \
    do {                                                                                           \
        if (A.packed && A.walls) RSPH_GO_PW(KERNEL, true, true, EV, __VA_ARGS__);                  \
        else if (A.packed) RSPH_GO_PW(KERNEL, true, false, EV, __VA_ARGS__);                       \
        else if (A.walls) RSPH_GO_PW(KERNEL, false, true, EV, __VA_ARGS__);                        \
        else RSPH_GO_PW(KERNEL, false, false, EV, __VA_ARGS__);                                    \
    } while (0)
// the colour pass takes the packed form only
#define RSPH_DISPATCH_PK(KERNEL, EV, ...)                                                          \
    do {                                                                                           \
        if (!A.packed) {                                                                           \
            RSPH_DISPATCH(KERNEL, G2, G3, EV, __VA_ARGS__);                                        \
        } else if (L.fp64) {                                                                       \
            if (L.dim == 2)                                                                        \
                go(KERNEL<double, 2, true>, slot_grid(A.P, G2), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
            else                                                                                   \
                go(KERNEL<double, 3, true>, slot_grid(A.P, G3), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
        } else {                                                                                   \
            if (L.dim == 2)                                                                        \
                go(KERNEL<float, 2, true>, slot_grid(A.P, G2), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
            else                                                                                   \
                go(KERNEL<float, 3, true>, slot_grid(A.P, G3), dim3(kBlock), L.stream, EV, __VA_ARGS__); \
        }                                                                                          \
    } while (0)

void launch_neighbours(const Launch& L, const DevArrays& A, Ev ev)
{
    RSPH_DISPATCH(k_neighbours, G2, G3, ev, A);
    if (L.dim == 3) {
        if (L.fp64)
            go(k_density<double, 3>, slot_grid(A.P, G3), dim3(kBlock), L.stream, Ev{}, A);
        else
            go(k_density<float, 3>, slot_grid(A.P, G3), dim3(kBlock), L.stream, Ev{}, A);
    }
}

int lanes_per_particle(int dim) { return dim == 2 ? G2 : G3; }

void launch_advection(const Launch& L, const DevArrays& A, Ev ev)
{
    RSPH_DISPATCH(k_advection, G2, G3, ev, A);
}

void launch_shift(const Launch& L, const DevArrays& A, Ev ev) { RSPH_DISPATCH(k_shift, G2, G3, ev, A); }

void launch_colour(const Launch& L, const DevArrays& A, Ev ev) { RSPH_DISPATCH_PK(k_colour, ev, A); }

void launch_force(const Launch& L, const DevArrays& A, Ev ev) { RSPH_DISPATCH_PW(k_force, ev, A); }

void launch_dt_substep(const Launch& L, const DevArrays& A, int64_t group)
{
    hipLaunchKernelGGL(k_dt_substep, dim3((unsigned)A.nsys), dim3(kBlock), 0, L.stream, A, group,
                       lanes_per_particle(L.dim));
}

void launch_continuity(const Launch& L, const DevArrays& A, Ev ev, int64_t group)
{
    RSPH_DISPATCH_PW(k_continuity, ev, A, group);
}

// ---------------------------------------------------------------------------
// device-resident particle input and rate output of the evaluation that works
// in the caller's device buffers (no staging through host memory)
// ---------------------------------------------------------------------------

// Particle i of the caller (row-major n x dim arrays on the device) into slot
// p_off + i: position wrapped into the box, velocity, mass (NULL: rho0 /
// sigma0), density (NULL: rho0), a zero continuity rate, caller index and
// fluid.  Inputs that the host could not check (a fluid outside {0, 1}, a
// non-finite value, a mass or density <= 0) set *bad; the fluid is then
// clamped so that every later index stays in bounds.
__global__ __launch_bounds__(kBlock) void k_load_particles(DevArrays A, int64_t p_off, int64_t n, int dim,
                                                           const double* pos, const double* vel,
                                                           const int32_t* phase, const double* mass,
                                                           const double* rho, double3 box, double2 rho0,
                                                           double sigma0, unsigned long long* probe)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t o = p_off + i;
    bool wrong = false;
    int ph = phase[i];
    if (ph != 0 && ph != 1 && ph != kWall) {
        wrong = true;
        ph = ph < 0 ? 0 : 1;
    }
    const double L[3] = {box.x, box.y, box.z};
    for (int a = 0; a < 3; ++a) {
        double q = a < dim ? pos[i * dim + a] : 0.0;
        const double v = a < dim ? vel[i * dim + a] : 0.0;
        wrong |= !isfinite(q) || !isfinite(v);
        if (a < dim) {
            q = q - L[a] * floor(q / L[a]);
            if (q >= L[a]) q -= L[a];
        }
        A.pos[a][o] = q;
        A.vel[a][o] = v;
    }
    const double r0 = ph == kWall ? 1.0 : (ph ? rho0.y : rho0.x);
    const double m = mass ? mass[i] : r0 / sigma0;
    const double r = rho ? rho[i] : r0;
    wrong |= !isfinite(m) || !(m > 0.0) || !isfinite(r) || !(r > 0.0);
    A.mass[o] = m;
    A.rho[o] = r;
    A.drho[o] = 0.0;
    A.id[o] = (int32_t)i;
    A.phase[o] = ph;
    if (wrong) atomicOr(probe, 1ull);
    if (ph == kWall) atomicOr(probe, 2ull);
    else if (!wrong) {
        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
        atomicMin(probe + 1 + ph, mb);
        atomicMax(probe + 3 + ph, mb);
    }
}

// Rates of the last evaluation, from slot order into the caller's order:
// acc (n x dim) and the continuity rate (n).
__global__ __launch_bounds__(kBlock) void k_store_rates(DevArrays A, int64_t p_off, int64_t n, int dim,
                                                        double* acc, double* drho)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t o = p_off + k;
    const int64_t id = A.id[o];
    for (int a = 0; a < dim; ++a) acc[id * dim + a] = A.r_acc[3 * o + a];
    drho[id] = A.r_drho[o];
}

void launch_load_particles(const Launch& L, const DevArrays& A, int64_t p_off, int64_t n, const double* pos,
                           const double* vel, const int32_t* phase, const double* mass, const double* rho,
                           const double* box, const double* rho0, double sigma0, unsigned long long* probe)
{
    if (n > 0)
        hipLaunchKernelGGL(k_load_particles, flat_grid(n), dim3(kBlock), 0, L.stream, A, p_off, n, L.dim, pos,
                           vel, phase, mass, rho, double3{box[0], box[1], box[2]}, double2{rho0[0], rho0[1]},
                           sigma0, probe);
}

void launch_store_rates(const Launch& L, const DevArrays& A, int64_t p_off, int64_t n, double* acc, double* drho)
{
    if (n > 0)
        hipLaunchKernelGGL(k_store_rates, flat_grid(n), dim3(kBlock), 0, L.stream, A, p_off, n, L.dim, acc, drho);
}

void launch_observables(const Launch& L, const DevArrays& A)
{
    const int64_t nwaves = A.P / kWave;
    for (int pass = 0; pass < 2; ++pass) {
        if (L.dim == 2)
            hipLaunchKernelGGL(k_obs_partial<2>, dim3((unsigned)nwaves), dim3(kWave), 0, L.stream, A, pass);
        else
            hipLaunchKernelGGL(k_obs_partial<3>, dim3((unsigned)nwaves), dim3(kWave), 0, L.stream, A, pass);
        hipLaunchKernelGGL(k_obs_final, dim3((unsigned)A.nsys), dim3(kBlock), 0, L.stream, A, pass);
    }
}

}  // namespace rsph
