// Device runtime of libswe.so: the fused stage kernel of the explicit
// shallow-water step (Delmas & Soulaimani, Sec. 6.1 - 6.2), the CFL
// reduction, ghost packing (Sec. 6.4) and the C ABI of include/swe.h.
//
// One thread per cell.  Cells are numbered in Morton order (send cells
// first), so a block's 1- and 2-ring gathers stay in the XCD's L2; blocks are
// remapped so that each of the 8 XCDs sweeps one contiguous range of tiles.
// Every interior edge flux is evaluated in the canonical orientation (L = the
// cell of smaller global id, L's normal) from identical operands wherever it
// is evaluated, so the two mass contributions cancel bitwise and results do
// not depend on the tiling; cell sums run over the local edges 0, 1, 2 in
// order; there are no atomics on the state, and the results are
// deterministic run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "swe_ctx.h"
#include "swe_mlp_dev.h"
#include "swe_internal.h"
#include "swe_kernels.h"

using namespace swe;

namespace {

constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;  // +inf as double bits

__device__ __forceinline__ unsigned long long dbits(double x)
{
    return (unsigned long long)__double_as_longlong(x);
}
__device__ __forceinline__ double bitsd(unsigned long long b)
{
    return __longlong_as_double((long long)b);
}

// Cross-lane moves by DPP (no LDS round trip).  CTRL is the DPP control:
// 0xB1 / 0x4E swap lanes within a quad (lane ^ 1, lane ^ 2), 0x124 / 0x128
// rotate a row of 16 lanes by 4 / 8, 0x142 / 0x143 broadcast lane 15 of a
// row to the next row / lane 31 to rows 2 and 3.  Rows outside ROWS keep
// `old`.  64-bit values move as two 32-bit halves.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp32(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS = 0xF, typename V>
__device__ __forceinline__ V dpp(V old, V v)
{
    static_assert(sizeof(V) == 4 || sizeof(V) == 8, "32- or 64-bit values");
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, dpp32<CTRL, ROWS>(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v)));
    } else {
        const int2 o = __builtin_bit_cast(int2, old), x = __builtin_bit_cast(int2, v);
        int2 r;
        r.x = dpp32<CTRL, ROWS>(o.x, x.x);
        r.y = dpp32<CTRL, ROWS>(o.y, x.y);
        return __builtin_bit_cast(V, r);
    }
}
template <typename V>
__device__ __forceinline__ V lane_value(V v, int lane)  // lane: the same in every lane
{
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
    } else {
        const int2 x = __builtin_bit_cast(int2, v);
        int2 r;
        r.x = __builtin_amdgcn_readlane(x.x, lane);
        r.y = __builtin_amdgcn_readlane(x.y, lane);
        return __builtin_bit_cast(V, r);
    }
}
template <typename V> __device__ __forceinline__ V vmin(V a, V b) { return a < b ? a : b; }
template <> __device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
template <> __device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
template <typename V> __device__ __forceinline__ V vmax(V a, V b) { return a > b ? a : b; }
template <> __device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
template <> __device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }

// Minimum and maximum over groups of g lanes (g = 1, 2, 4, 8 or 16) when
// every group of a row of 16 lanes holds the same g values: afterwards every
// lane holds the group's minimum and maximum.  (With g = 8 the rotation by 4
// joins a group's half with the other group's opposite half: the same
// values.)  Every lane of the wave takes part.  min and max are exact, so
// the order of the steps does not change the result.
template <typename V>
__device__ __forceinline__ void group_minmax(V &mn, V &mx, int g)
{
    if (g > 1) { mn = vmin(mn, dpp<0xB1>(mn, mn)); mx = vmax(mx, dpp<0xB1>(mx, mx)); }
    if (g > 2) { mn = vmin(mn, dpp<0x4E>(mn, mn)); mx = vmax(mx, dpp<0x4E>(mx, mx)); }
    if (g > 4) { mn = vmin(mn, dpp<0x124>(mn, mn)); mx = vmax(mx, dpp<0x124>(mx, mx)); }
    if (g > 8) { mn = vmin(mn, dpp<0x128>(mn, mn)); mx = vmax(mx, dpp<0x128>(mx, mx)); }
}

// Minimum and maximum over the 64 lanes of the wave, returned in every lane
// (every lane takes part).
template <typename V>
__device__ __forceinline__ void wave_minmax(V &mn, V &mx)
{
    group_minmax(mn, mx, 16);
    mn = vmin(mn, dpp<0x142, 0xA>(mn, mn));
    mx = vmax(mx, dpp<0x142, 0xA>(mx, mx));
    mn = vmin(mn, dpp<0x143, 0xC>(mn, mn));
    mx = vmax(mx, dpp<0x143, 0xC>(mx, mx));
    mn = lane_value(mn, 63);
    mx = lane_value(mx, 63);
}

__device__ __forceinline__ int xcd_tile(int bid, int nb)
{
    // blocks are dealt to the 8 XCDs round-robin; give XCD x one contiguous
    // range of tiles so that neighbouring tiles share its L2
    const int x = bid & 7, i = bid >> 3, base = nb >> 3, rem = nb & 7;
    return x * base + (x < rem ? x : rem) + i;
}

using ClockWord = unsigned long long;

// First word of clock slot `slot` of scenario s (the time); copy j of the
// CFL partials starts kClockLine * (1 + j) words further.
__host__ __device__ inline size_t clock_off(int ncopy, int s, int slot)
{
    return (size_t)(3 * s + slot) * (size_t)(ncopy + 1) * kClockLine;
}

// The CFL step (Sec. 6.2) from the reduced quantities; dt_max when nothing
// is wet (no cell committed).
__device__ __forceinline__ double cfl_dt(double mn, double mx, double cfl, double dt_max, int rule)
{
    if (!(mn < __builtin_huge_val())) return dt_max > 0.0 ? dt_max : 0.0;
    double dt = rule == 1 ? cfl * mn / mx : cfl * mn;
    if (dt_max > 0.0 && dt > dt_max) dt = dt_max;
    return dt;
}

// Step of scenario s whose CFL partials are in clock slot `slot` (dt_fixed
// when positive).  Every lane of the wave calls it; lanes with s < 0 get 0.
// For each distinct scenario of the wave the copies are loaded one per lane
// and reduced with shuffles, so all lanes agree bitwise.
__device__ __forceinline__ double wave_step_dt(const ClockWord *clk, int ncopy, int slot, int s,
                                               int rule, double cfl, double dt_max, double dt_fixed)
{
    if (dt_fixed > 0.0) return dt_fixed;
    const int lane = threadIdx.x & 63;
    double dt = 0.0;
    bool have = s < 0;
    for (;;) {
        const unsigned long long pend = __ballot(!have);
        if (pend == 0ull) break;
        const int S = lane_value(s, __builtin_ctzll(pend));
        // every group of ncopy lanes loads all copies, so the reduction
        // within the group leaves the full result in every lane
        const ClockWord *q =
            clk + clock_off(ncopy, S, slot) + (size_t)(1 + (lane & (ncopy - 1))) * kClockLine;
        double mn = bitsd(q[kCfqMin]), mx = bitsd(q[kCfqMax]);
        group_minmax(mn, mx, ncopy);
        if (s == S) {
            dt = cfl_dt(mn, mx, cfl, dt_max, rule);
            have = true;
        }
    }
    return dt;
}

// The step in two halves, so that the latency of the clock lines (last
// written by atomics of the previous kernel) hides behind the stencil work:
// dt_prefetch loads, per lane, copy (lane mod ncopy) of the partials of the
// scenario of the wave's first cell; dt_finish reduces them when the wave's
// cells all belong to that scenario and otherwise falls back to
// wave_step_dt.  Every lane of the wave calls both.
struct DtPrefetch {
    double mn, mx;
    int S;
};

__device__ __forceinline__ DtPrefetch dt_prefetch(const ClockWord *clk, int ncopy, int slot,
                                                  int s_own, double dt_fixed)
{
    DtPrefetch p;
    const unsigned long long act = __ballot(s_own >= 0);
    p.S = act ? lane_value(s_own, __builtin_ctzll(act)) : 0;
    p.mn = 0.0;
    p.mx = 0.0;
    if (dt_fixed <= 0.0) {
        const ClockWord *q = clk + clock_off(ncopy, p.S, slot) +
                             (size_t)(1 + ((int)threadIdx.x & (ncopy - 1))) * kClockLine;
        p.mn = bitsd(q[kCfqMin]);
        p.mx = bitsd(q[kCfqMax]);
    }
    return p;
}

__device__ __forceinline__ double dt_finish(DtPrefetch p, const ClockWord *clk, int ncopy, int slot,
                                            int s, int rule, double cfl, double dt_max,
                                            double dt_fixed)
{
    if (dt_fixed > 0.0) return dt_fixed;
    if (__ballot(s >= 0 && s != p.S) != 0ull)
        return wave_step_dt(clk, ncopy, slot, s, rule, cfl, dt_max, dt_fixed);
    group_minmax(p.mn, p.mx, ncopy);
    return s >= 0 ? cfl_dt(p.mn, p.mx, cfl, dt_max, rule) : 0.0;
}

// The same step as wave_step_dt for one lane on its own (copies reduced in
// a loop; min and max are exact, so both agree bitwise).  For rare
// divergent paths.
__device__ __forceinline__ double lane_step_dt(const ClockWord *clk, int ncopy, int slot, int s,
                                               int rule, double cfl, double dt_max, double dt_fixed)
{
    if (dt_fixed > 0.0) return dt_fixed;
    const ClockWord *q = clk + clock_off(ncopy, s, slot) + kClockLine;
    double mn = bitsd(q[kCfqMin]), mx = bitsd(q[kCfqMax]);
    for (int j = 1; j < ncopy; ++j) {
        mn = fmin(mn, bitsd(q[(size_t)j * kClockLine + kCfqMin]));
        mx = fmax(mx, bitsd(q[(size_t)j * kClockLine + kCfqMax]));
    }
    return cfl_dt(mn, mx, cfl, dt_max, rule);
}

// Per-cell CFL quantities (Sec. 6.2) of a wet owned cell, in the working
// precision: mn = R_i / lambda_i (rule 0) or R_i (rule 1), mx = lambda_i;
// neutral values otherwise.  They become doubles only when committed (the
// conversion is monotonic, so reducing before or after it agrees).
template <typename T> struct CflVal {
    T mn, mx;
    int scen;  // -1: no cell
};

template <typename T> __device__ __forceinline__ CflVal<T> cfl_none()
{
    CflVal<T> v;
    v.mn = T(__builtin_huge_val());
    v.mx = T(0);
    v.scen = -1;
    return v;
}

template <typename T> __device__ __forceinline__ CflVal<T> cfl_cell(int rule, int scen, T R, T lam)
{
    CflVal<T> v;
    v.mn = rule == 1 ? R : fdiv(R, lam);
    v.mx = lam;
    v.scen = scen;
    return v;
}

// One commit of a block's (or lane's) partial: min mn always, max mx only
// where the step rule reads it.
template <typename T>
__device__ __forceinline__ void cfl_atomic(ClockWord *q, int rule, const CflVal<T> &v)
{
    atomicMin(&q[kCfqMin], dbits(double(v.mn)));
    if (rule == 1) atomicMax(&q[kCfqMax], dbits(double(v.mx)));
}

// Block-wide reduction of the CFL quantities into clock slot `slot` of each
// scenario: shuffles within each wave, the wave results through LDS, then
// one thread commits one set of atomics per run of waves of the same
// scenario (one set per block unless the block straddles two scenarios of a
// batch; a wave that itself straddles commits per lane), to the block's
// copy of the partials.  Same-address device atomics serialise, so their
// number per address, not the cell work, would otherwise bound the stage.
// Every thread of the block calls this; `part` holds one entry per wave and
// may be reused after the next __syncthreads().
template <typename T>
__device__ __forceinline__ void cfl_commit(ClockWord *clk, int ncopy, int slot, int rule,
                                           CflVal<T> v, CflVal<T> *part)
{
    const size_t copy = (size_t)(1 + (blockIdx.x & (ncopy - 1))) * kClockLine;
    int smin = v.scen >= 0 ? v.scen : 0x7fffffff, smax = v.scen;
    wave_minmax(smin, smax);
    if (smin == smax) {
        wave_minmax(v.mn, v.mx);
        v.scen = smax;
    } else {
        if (v.scen >= 0 && v.mx > T(0)) cfl_atomic(clk + clock_off(ncopy, v.scen, slot) + copy, rule, v);
        v.scen = -1;
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = ((int)blockDim.x + 63) >> 6;
        CflVal<T> run = cfl_none<T>();
        for (int w = 0; w < nw; ++w) {
            const CflVal<T> p = part[w];
            if (p.scen < 0 || !(p.mx > T(0))) continue;
            if (p.scen != run.scen) {
                if (run.scen >= 0) cfl_atomic(clk + clock_off(ncopy, run.scen, slot) + copy, rule, run);
                run = p;
            } else {
                run.mn = fmin(run.mn, p.mn);
                run.mx = fmax(run.mx, p.mx);
            }
        }
        if (run.scen >= 0) cfl_atomic(clk + clock_off(ncopy, run.scen, slot) + copy, rule, run);
    }
}

// Total inflow discharge at time t: the scenario's hydrograph, linear
// between its points and held constant outside them, else its constant.
__device__ __forceinline__ double inflow_at(const ScenParams &s, const double *ts, const double *qs,
                                            double t)
{
    if (s.series_n <= 0) return s.inflow_q;
    const double *T = ts + s.series_off, *Q = qs + s.series_off;
    const int n = s.series_n;
    if (t <= T[0]) return Q[0];
    if (t >= T[n - 1]) return Q[n - 1];
    for (int i = 0; i + 1 < n; ++i)
        if (t <= T[i + 1]) return Q[i] + (Q[i + 1] - Q[i]) * (t - T[i]) / (T[i + 1] - T[i]);
    return Q[n - 1];
}

template <typename T> struct StageArgs {
    using T4 = typename V4<T>::type;
    int n, n_scen;
    const int4 *nbr;
    const T4 *cell, *he_geo, *he_dist;
    const T *man2;  // Manning n^2 per cell (tiled MUSCL kernel: its only per-cell record)
    // per half-edge, edge-major (m * n + c): nx, ny, d_mid / d_up, d_mid / d_fwd;
    // L / area; d_mid / d_central
    const T4 *he_co;
    const T *he_lam, *he_gam;
    const T *he_dfw;  // tiled WAF: centroid distance d_fwd per half-edge (edge-major)
    const typename V2<T>::type *he_nrm;  // tiled WAF: unit normal per half-edge (edge-major)
    const T4 *Uin, *U0;
    T4 *Uout;
    ClockWord *clock;
    int ncopy;                   // CFL partial copies per clock slot (power of two <= 64)
    const ScenParams *scen;
    const double *ser_t, *ser_q;
    // learned limiter: phi per half-edge (3 c + m), stored by the instance
    // of the tiled stage that evaluates the network (the step's first
    // stage), read by the others
    float *phi;
    const MlpDev *mlp;
    int *health;
    T g, eps;
    int waf_pos;  // WAF: mass fluxes kept within the donor cells' shares (waf_positivity)
    double cfl, dt_max, dt_fixed;
    int slot_cur, slot_next, slot_reset;
    int kind;  // 0: Euler step, 1: first RK2 stage, 2: second RK2 stage (+ average)
    int cfl_rule;
    // fused pack of the high-overlap step (last stage only; pk_buf null
    // otherwise): the new state of send cell c < pk_ncell goes to the send
    // entries pk_ent[pk_off[c] .. pk_off[c+1]) of pk_buf ([3][pk_nsend])
    const int *pk_off, *pk_ent;
    T *pk_buf;
    int pk_ncell, pk_nsend;
};

// Fused pack: the thread that has just computed send cell c's new state
// writes it to every send entry of c (bitwise the stored state).
template <typename T>
__device__ __forceinline__ void pack_own(const StageArgs<T> &a, int c, T nh, T nu, T nv)
{
    if (a.pk_buf == nullptr || c >= a.pk_ncell) return;
    const int e1 = a.pk_off[c + 1];
    for (int e = a.pk_off[c]; e < e1; ++e) {
        const int j = a.pk_ent[e];
        a.pk_buf[j] = nh;
        a.pk_buf[a.pk_nsend + j] = nu;
        a.pk_buf[2 * a.pk_nsend + j] = nv;
    }
}

// Boundary flux of Sec. 6.1 in the global frame.
template <typename T, typename T4>
__device__ __forceinline__ void boundary_flux(int tag, const T4 &Uc, T nx, T ny, T g, T eps, T q_in,
                                              T stage, T G[3])
{
    const T h = Uc.x;
    T U[3] = {h, Uc.y * nx + Uc.z * ny, -Uc.y * ny + Uc.z * nx};
    T F[3];
    if (tag == kBcWall) {
        F[0] = T(0); F[1] = T(0.5) * g * h * h; F[2] = T(0);
    } else if (tag == kBcInflow) {
        const T hl = tmax(h, T(1e-3));
        F[0] = -q_in; F[1] = fdiv(q_in * q_in, hl) + T(0.5) * g * h * h; F[2] = T(0);
    } else if (tag == kBcOutflow) {
        const T hg = tmax(T(0), stage - Uc.w);
        const T un = h > eps ? fdiv(U[1], h) : T(0), ut = h > eps ? fdiv(U[2], h) : T(0);
        T UG[3] = {hg, hg * un, hg * ut};
        flux_hllc(g, eps, U, UG, F);
    } else {
        flux_hllc(g, eps, U, U, F);
    }
    G[0] = F[0];
    G[1] = F[1] * nx - F[2] * ny;
    G[2] = F[1] * ny + F[2] * nx;
}

// Boundary flux of Sec. 6.1 in the global frame, less the hydrostatic
// pressure g h^2 / 2 of the cell along the normal (the pressure-deviation
// form of the tiled kernel): a wall then contributes nothing.
template <typename T, typename T4>
__device__ __forceinline__ void boundary_flux_dev(int tag, const T4 &Uc, T nx, T ny, T g, T eps,
                                                  T q_in, T stage, T G[3])
{
    const T h = Uc.x;
    T F0 = T(0), D = T(0), F2 = T(0);
    if (tag == kBcInflow) {
        const T hl = tmax(h, T(1e-3));
        F0 = -q_in;
        D = fdiv(q_in * q_in, hl);
    } else if (tag != kBcWall) {
        const T r = h > eps ? frcp(h) : T(0);
        const T un = (Uc.y * nx + Uc.z * ny) * r, ut = (-Uc.y * ny + Uc.z * nx) * r;
        const T hg = tag == kBcOutflow ? tmax(T(0), stage - Uc.w) : h;
        T DR;
        hllc_dev(g, eps, h, un, ut, hg, un, ut, F0, D, DR, F2);
    }
    G[0] = F0;
    G[1] = D * nx - F2 * ny;
    G[2] = D * ny + F2 * nx;
}

template <typename T, typename T4>
__device__ __forceinline__ T tangential(const T4 &U, T nx, T ny, T eps)
{
    return U.x > eps ? fdiv(-U.y * ny + U.z * nx, U.x) : T(0);
}

// upwind mean of eta and v (L frame) over a cell's two upwind neighbours; a
// missing or dry neighbour does not count
template <typename T, typename T4>
__device__ __forceinline__ bool waf_upwind(const T4 &Ua, bool ha, const T4 &Ub, bool hb, T nx,
                                           T ny, T eps, T &e, T &v)
{
    ha = ha && Ua.x > eps;
    hb = hb && Ub.x > eps;
    if (ha && hb) {
        e = T(0.5) * ((Ua.x + Ua.w) + (Ub.x + Ub.w));
        v = T(0.5) * (tangential(Ua, nx, ny, eps) + tangential(Ub, nx, ny, eps));
    } else if (ha) {
        e = Ua.x + Ua.w; v = tangential(Ua, nx, ny, eps);
    } else if (hb) {
        e = Ub.x + Ub.w; v = tangential(Ub, nx, ny, eps);
    } else {
        e = T(0); v = T(0);
    }
    return ha || hb;
}

// Element i of an array addressed with a 32-bit byte offset from a uniform
// base (the arrays of a context stay below 4 GiB, checked at upload), so
// the load takes one offset register and no 64-bit address arithmetic.
template <typename V> __device__ __forceinline__ V ldx(const V *base, unsigned i)
{
    return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + i * (unsigned)sizeof(V));
}
template <typename V> __device__ __forceinline__ void stx(V *base, unsigned i, const V &v)
{
    *reinterpret_cast<V *>(reinterpret_cast<char *>(base) + i * (unsigned)sizeof(V)) = v;
}

// Component m (0..2) of an int4 by selects (no local array: a dynamically
// indexed one lives in scratch memory).
__device__ __forceinline__ int pick3(const int4 &v, int m)
{
    return m == 0 ? v.x : (m == 1 ? v.y : v.z);
}

// Clock upkeep of a stage kernel: the first kernel of a step clears the
// partials of slot step + 2 (spread over the grid); the last one advances
// each scenario's time by its step (wave 0 of block s mod grid).
template <typename T>
__device__ __forceinline__ void clock_upkeep(const StageArgs<T> &a)
{
    if (a.kind != 2) {
        const int ne = a.n_scen * a.ncopy;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
            ClockWord *q = a.clock + clock_off(a.ncopy, e / a.ncopy, a.slot_reset) +
                           (size_t)(1 + e % a.ncopy) * kClockLine;
            q[kCfqMin] = kInfBits;
            q[kCfqMax] = 0ull;
        }
    }
    if (a.kind != 1 && threadIdx.x < 64) {
        for (int s = blockIdx.x; s < a.n_scen; s += gridDim.x) {
            const double dt = wave_step_dt(a.clock, a.ncopy, a.slot_cur, s, a.cfl_rule, a.cfl,
                                           a.dt_max, a.dt_fixed);
            if (threadIdx.x == 0)
                a.clock[clock_off(a.ncopy, s, a.slot_next)] =
                    dbits(bitsd(a.clock[clock_off(a.ncopy, s, a.slot_cur)]) + dt);
        }
    }
}

// One cell of one stage (all of Sec. 6.1 - 6.2 for cell c); returns the
// cell's CFL quantities for the next step.
template <typename T, int SCHEME, int LIM, int WAFM>
__device__ __forceinline__ CflVal<T> stage_cell(const StageArgs<T> &a, const int c)
{
    using T4 = typename V4<T>::type;
    CflVal<T> cfl = cfl_none<T>();
    int4 nb4 = make_int4(-1, -1, -1, 0);
    int s = -1;
    if (c < a.n) {
        nb4 = a.nbr[c];
        s = (int)((unsigned)nb4.w >> kScenShift);
    }
    const double dtd =
        wave_step_dt(a.clock, a.ncopy, a.slot_cur, s, a.cfl_rule, a.cfl, a.dt_max, a.dt_fixed);
    if (c < a.n) {
        const unsigned word = (unsigned)nb4.w;
        const T dt = T(dtd);
        const T g = a.g, eps = a.eps;
        const T4 Uc = a.Uin[c];
        const T4 cg = a.cell[c];
        // neighbours in separate variables, picked by selects: a local
        // array indexed at run time would live in scratch memory
        const int nb0 = nb4.x, nb1 = nb4.y, nb2 = nb4.z;
        const bool hn0 = nb0 >= 0, hn1 = nb1 >= 0, hn2 = nb2 >= 0;
        // (the index is selected, not the value: a select between a load and
        // a local value becomes a load through a selected pointer, which
        // puts the local value in scratch memory)
        const T4 Un0 = a.Uin[hn0 ? nb0 : c], Un1 = a.Uin[hn1 ? nb1 : c], Un2 = a.Uin[hn2 ? nb2 : c];
        T acc0 = T(0), acc1 = T(0), acc2 = T(0);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T4 ge = a.he_geo[3 * c + m];
            const T nx = ge.x, ny = ge.y, L = ge.z;
            const int k = m == 0 ? nb0 : (m == 1 ? nb1 : nb2);
            if (k < 0) {
                const ScenParams sp = a.scen[s];
                const double t_st =
                    bitsd(a.clock[clock_off(a.ncopy, s, a.slot_cur)]) + (a.kind == 2 ? dtd : 0.0);
                const T q_in = k == kBcInflow
                                   ? T(inflow_at(sp, a.ser_t, a.ser_q, t_st) * sp.inv_inflow_len)
                                   : T(0);
                T G[3];
                boundary_flux<T, T4>(k, Uc, nx, ny, g, eps, q_in, T(sp.outflow_stage), G);
                acc0 += L * G[0];
                acc1 += L * G[1];
                acc2 += L * G[2];
                continue;
            }
            const int ma = (m + 1) % 3, mb = (m + 2) % 3;
            const T4 Um = m == 0 ? Un0 : (m == 1 ? Un1 : Un2);
            const T4 Ua = ma == 0 ? Un0 : (ma == 1 ? Un1 : Un2);
            const T4 Ub = mb == 0 ? Un0 : (mb == 1 ? Un1 : Un2);
            const bool ha = ma == 0 ? hn0 : (ma == 1 ? hn1 : hn2);
            const bool hb = mb == 0 ? hn0 : (mb == 1 ? hn1 : hn2);
            const int jb = (word >> (2 * m)) & 3;
            T4 zero4;
            zero4.x = T(0); zero4.y = T(0); zero4.z = T(0); zero4.w = T(0);
            T4 Uka = Uc, Ukb = Uc;
            bool hka = false, hkb = false;
            if (SCHEME != kHLLC1) {
                const int4 nk = a.nbr[k];
                const int ka = pick3(nk, (jb + 1) % 3), kb = pick3(nk, (jb + 2) % 3);
                hka = ka >= 0;
                hkb = kb >= 0;
                if (hka) Uka = a.Uin[ka];
                if (hkb) Ukb = a.Uin[kb];
            }
            T4 dc = zero4, dk = zero4;
            T dmk = T(0);
            float phic = 0.0f, phik = 0.0f;
            if (SCHEME == kMUSCL) {
                dc = a.he_dist[3 * c + m];
                dk = a.he_dist[3 * k + jb];
                dmk = a.he_geo[3 * k + jb].w;
                if (LIM == kLearned) { phic = a.phi[3 * c + m]; phik = a.phi[3 * k + jb]; }
            }
            const Half<T> own = reconstruct<T, T4, SCHEME, LIM>(Uc, Um, Ua, ha, Ub, hb, nx, ny, ge.w,
                                                                dc, phic, eps);
            const Half<T> oth = reconstruct<T, T4, SCHEME, LIM>(Um, Uc, Uka, hka, Ukb, hkb, -nx,
                                                                -ny, dmk, dk, phik, eps);
            // hydrostatic reconstruction
            const T be = tmax(own.b, oth.b);
            const T hso = tmax(T(0), own.h + own.b - be);
            const T hsk = tmax(T(0), oth.h + oth.b - be);
            const bool isL = (word >> (6 + m)) & 1u;
            T UL[3], UR[3];
            T nLx, nLy;
            if (isL) {
                UL[0] = hso; UL[1] = hso * own.un; UL[2] = hso * own.ut;
                UR[0] = hsk; UR[1] = -(hsk * oth.un); UR[2] = -(hsk * oth.ut);
                nLx = nx; nLy = ny;
            } else {
                UL[0] = hsk; UL[1] = hsk * oth.un; UL[2] = hsk * oth.ut;
                UR[0] = hso; UR[1] = -(hso * own.un); UR[2] = -(hso * own.ut);
                nLx = -nx; nLy = -ny;
            }
            T F[3];
            if (SCHEME == kWAF) {
                const T4 dw = a.he_dist[3 * c + m];
                // values, not references: a reference chosen at run time
                // would put both states in scratch memory
                const T4 ULc = isL ? Uc : Um;
                const T4 URc = isL ? Um : Uc;
                WafIn<T> w;
                w.eL = ULc.x + ULc.w; w.eR = URc.x + URc.w;
                w.vL = tangential(ULc, nLx, nLy, eps);
                w.vR = tangential(URc, nLx, nLy, eps);
                T eo, vo, ek, vk;
                const bool ho = waf_upwind(Ua, ha, Ub, hb, nLx, nLy, eps, eo, vo);
                const bool hk = waf_upwind(Uka, hka, Ukb, hkb, nLx, nLy, eps, ek, vk);
                if (isL) { w.eLu = eo; w.vLu = vo; w.hasLu = ho; w.eRu = ek; w.vRu = vk; w.hasRu = hk; }
                else { w.eLu = ek; w.vLu = vk; w.hasLu = hk; w.eRu = eo; w.vRu = vo; w.hasRu = ho; }
                flux_waf<T, WAFM>(g, eps, fdiv(dt, dw.w), UL, UR, w, F);
                if (a.waf_pos) {
                    const T Rc = cg.y, Rk = ((const T *)a.cell)[4 * (size_t)k + 1];
                    waf_positivity(g, eps, UL, UR, isL ? Uc.x : Um.x, isL ? Rc : Rk, isL ? Um.x : Uc.x,
                                   isL ? Rk : Rc, dt, F);
                }
            } else {
                flux_hllc(g, eps, UL, UR, F);
            }
            const T G0 = F[0];
            const T G1 = F[1] * nLx - F[2] * nLy;
            const T G2 = F[1] * nLy + F[2] * nLx;
            const T sg = isL ? T(1) : T(-1);
            const T p = T(0.5) * g * (own.h * own.h - hso * hso);  // side correction
            const T sb = T(0.5) * g * (own.h + Uc.x) * (own.b - Uc.w);  // centred bed term
            acc0 += L * (sg * G0);
            acc1 += L * (sg * G1 + (p + sb) * nx);
            acc2 += L * (sg * G2 + (p + sb) * ny);
        }
        T nh = Uc.x - dt * (acc0 * cg.x);
        T nu = Uc.y - dt * (acc1 * cg.x);
        T nv = Uc.z - dt * (acc2 * cg.x);
        int flags = 0;
        if (!(isfinite(nh) && isfinite(nu) && isfinite(nv))) flags |= kHealthNonfinite;
        if (nh < T(0)) {
            flags |= nh < -eps ? kHealthNegDepth : kHealthClipped;
            nh = T(0);
        }
        if (nh <= eps) {
            nu = T(0); nv = T(0);
        } else if (cg.z > T(0)) {  // Manning, point-implicit
            const T sp = fdiv(sqrt(nu * nu + nv * nv), nh);
            const T f = T(1) + dt * g * cg.z * sp * pow_m43(nh);
            { const T rf = frcp(f); nu *= rf; nv *= rf; }
        }
        if (a.kind == 2) {  // SSP-RK2: average with U^n
            const T4 U0c = a.U0[c];
            nh = T(0.5) * (U0c.x + nh);
            nu = T(0.5) * (U0c.y + nu);
            nv = T(0.5) * (U0c.z + nv);
            if (nh <= eps) { nu = T(0); nv = T(0); }
        }
        T4 out;
        out.x = nh; out.y = nu; out.z = nv; out.w = Uc.w;
        a.Uout[c] = out;
        pack_own(a, c, nh, nu, nv);
        // health counts owned cells: a ghost cell's new state is provisional
        // (the next exchange replaces it)
        if (flags && ((word >> kOwnedBit) & 1u)) atomicOr(a.health, flags);
        cfl.scen = s;
        if (a.kind != 1 && ((word >> kOwnedBit) & 1u) && nh > eps) {
            const T u = fdiv(nu, nh), v = fdiv(nv, nh);
            const T lm = sqrt(u * u + v * v) + sqrt(g * nh);
            cfl = cfl_cell<T>(a.cfl_rule, s, cg.y, lm);
        }
    }
    return cfl;
}

template <typename T, int SCHEME, int LIM, int WAFM>
__global__ void __launch_bounds__(256) k_stage(StageArgs<T> a)
{
    clock_upkeep(a);
    // one tile per block, or (persistent launch, gridDim < tiles) a
    // grid-stride sweep; either way each XCD takes contiguous tiles
    __shared__ CflVal<T> part[4];
    const int ntiles = (a.n + (int)blockDim.x - 1) / (int)blockDim.x;
    for (int t = xcd_tile(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x) {
        const CflVal<T> v = stage_cell<T, SCHEME, LIM, WAFM>(a, t * (int)blockDim.x + (int)threadIdx.x);
        if (a.kind != 1) {
            cfl_commit(a.clock, a.ncopy, a.slot_next, a.cfl_rule, v, part);
            __syncthreads();  // part is reused by the next tile
        }
    }
}

// ------------------------------------------------------------------------
// Tiled stage kernel (first-order HLLC and MUSCL-HLLC).  A block owns one
// tile of TILE consecutive (Morton-ordered) cells:
//  1. every thread forms the primitive values of its cell and its 1-ring,
//     reconstructs its interior half-edges into LDS (with the centred bed
//     term of each), and files its edges as tasks: an edge to a cell of the
//     same tile is filed once, by the cell that is the L side of the
//     canonical orientation; an edge to a cell outside the tile is filed by
//     each side;
//  2. the block sweeps both task lists as one dense range (outside edges
//     first: they also reconstruct the far side from its 2-ring; then inside
//     edges, whose far side is already in LDS): hydrostatic reconstruction,
//     HLLC in the canonical orientation, side corrections; each half-edge's
//     share replaces its interface values in LDS (a slot is read and written
//     by one task only);
//  3. every thread sums its three half-edge shares weighted by L / area,
//     updates, applies Manning and the cleanup, and the block commits its
//     CFL quantities.
// Boundary half-edges are tasks of the first list too (their flux needs
// only the cell's own state).
// The flux of an edge is the same function of the same operands wherever it
// is evaluated (operands selected, one evaluation, multiply-adds fused per
// expression only), so results do not depend on the tiling (sub-domain runs
// stay bitwise equal to undecomposed runs) and mass contributions cancel
// bitwise.  Momentum is summed in pressure-deviation form: every share of a
// cell is taken less the cell's own hydrostatic pressure g h^2 / 2 along its
// normal, which changes nothing exactly (the outward normals of a triangle
// times its edge lengths sum to zero) but makes a lake at rest exactly at
// rest in floating point and removes the rounding of the large cancelling
// pressure terms (Sec. 6.2.3's side corrections and centred bed term become
// g (h- + h)(eta- - eta) / 2; hllc_dev gives F1 - g h*^2 / 2 per side).
// LDS per cell: 3 x (4 + 1) values, 3 task slots, 3 neighbour indices and
// the word (22.5 KB per 256-cell FP32 tile, seven tiles per CU); phase 2
// reads no global memory for edges inside the tile but the normal.  Half-edge
// slots are local-edge-major (slot of cell l, edge m at m * TILE + l), so a
// wave's per-cell accesses are consecutive.
// Learned limiter in the step's first stage: the tiled instance that also
// evaluates the network and stores phi (the second stage reads it)
constexpr int kLearnedNet = 5;
#ifndef SWE_TILED_WAVES
#define SWE_TILED_WAVES 6  // FP32: waves per SIMD the register budget is sized for
#endif
#ifndef SWE_TILED_WAVES_LEARNED
#define SWE_TILED_WAVES_LEARNED 5  // the learned-limiter instance needs 96 registers
#endif
#ifndef SWE_TILED_WAVES_NET
#define SWE_TILED_WAVES_NET 4  // the instance that also evaluates the network (128 registers)
#endif
template <typename T, bool MUSCL_, int LIM, int TILE, int OCC = SWE_TILED_WAVES>
__global__ void __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 ? (LIM == kLearned ? SWE_TILED_WAVES_LEARNED
                                      : (LIM == kLearnedNet ? SWE_TILED_WAVES_NET : OCC))
                   : 2)))
k_stage_tiled(StageArgs<T> a)
{
    using T4 = typename V4<T>::type;
    static_assert(TILE <= 1024, "10-bit tile-local indices in task entries");
    __shared__ T4 sR[3 * TILE];
    __shared__ T sB[3 * TILE];
    // tasks: outside-tile and boundary half-edges from the front, inside
    // edges from the back; an entry packs m (2 bits), the filing cell (10),
    // the neighbour's local edge jb (2), the L-side bit and, inside the
    // tile, the neighbour's tile-local index (10)
    __shared__ unsigned sTask[3 * TILE];
    __shared__ int sK[3 * TILE];       // neighbour (or boundary tag) of each half-edge
    __shared__ unsigned sW[TILE];      // packed word of each cell
    __shared__ int sCount[2];
    __shared__ CflVal<T> sCfl[TILE / 64];
    // learned limiter: kNet evaluates phi (input rows of the network in LDS,
    // 64 per wave), kLrn reads it; RL is the limiter of the reconstruction
    constexpr bool kNet = MUSCL_ && LIM == kLearnedNet;
    constexpr bool kLrn = MUSCL_ && (LIM == kLearned || LIM == kLearnedNet);
    constexpr int RL = LIM == kLearnedNet ? kLearned : LIM;
    __shared__ __align__(16) uint16_t sX[kNet ? TILE : 1][16];
    clock_upkeep(a);
    const T g = a.g, eps = a.eps;
    const int ntiles = (a.n + TILE - 1) / TILE;
    for (int tile = xcd_tile(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
        const int c0 = tile * TILE, cl = threadIdx.x, c = c0 + cl;
        const bool active = c < a.n;
        if (threadIdx.x < 2) sCount[threadIdx.x] = 0;
        __syncthreads();
        // a tile's first phase issues its chains of dependent loads (the
        // neighbour quads, then the stencil): waves in it go first, ahead
        // of waves sweeping edges or updating (measured: 1.8% on the
        // 13M-cell river, 2.2% with the update's priority below, even on
        // config 2; the WAF kernel gains nothing)
        __builtin_amdgcn_s_setprio(3);
        // ---- 1: primitives, own half-edges, task lists
        DtPrefetch dtp;
        int4 nb4 = make_int4(-1, -1, -1, 0);
        if (active) nb4 = ldx(a.nbr, c);
        dtp = dt_prefetch(a.clock, a.ncopy, a.slot_cur, active ? (int)((unsigned)nb4.w >> kScenShift) : -1,
                          a.dt_fixed);
        T4 Ukeep;  // the cell's state, kept for phase 3
        if constexpr (kLrn) {
            // phi of the cell's three half-edges: in the step's first stage
            // from the network on U^n (the wave evaluates its 64 half-edges
            // of one local edge at a time) and stored for the second, else
            // the stored values
            const bool hn0 = active && nb4.x >= 0, hn1 = active && nb4.y >= 0, hn2 = active && nb4.z >= 0;
            float ph[3] = {0.0f, 0.0f, 0.0f};
            if constexpr (kNet) {
                T4 Uc{}, Un0{}, Un1{}, Un2{}, co0{}, co1{}, co2{};
                if (active) {
                    Uc = ldx(a.Uin, c);
                    Un0 = ldx(a.Uin, hn0 ? nb4.x : c);
                    Un1 = ldx(a.Uin, hn1 ? nb4.y : c);
                    Un2 = ldx(a.Uin, hn2 ? nb4.z : c);
                    co0 = ldx(a.he_co, c);
                    co1 = ldx(a.he_co, a.n + c);
                    co2 = ldx(a.he_co, 2 * a.n + c);
                }
                const int lane = threadIdx.x & 63;
                uint16_t(*X)[16] = sX + (threadIdx.x & ~63);
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const int ma = (m + 1) % 3, mb = (m + 2) % 3;
                    const T4 Um = m == 0 ? Un0 : (m == 1 ? Un1 : Un2);
                    const T4 Ua = ma == 0 ? Un0 : (ma == 1 ? Un1 : Un2);
                    const T4 Ub = mb == 0 ? Un0 : (mb == 1 ? Un1 : Un2);
                    const bool hm = m == 0 ? hn0 : (m == 1 ? hn1 : hn2);
                    const bool ha = ma == 0 ? hn0 : (ma == 1 ? hn1 : hn2);
                    const bool hb = mb == 0 ? hn0 : (mb == 1 ? hn1 : hn2);
                    const T4 co = m == 0 ? co0 : (m == 1 ? co1 : co2);
                    float f[kMlpIn];
                    const bool ok = limiter_features<T, T4>(Uc, Um, hm, Ua, ha, Ub, hb, co.x, co.y,
                                                            co.z, co.w, g, eps, f);
                    mlp_write_row(X[lane], f, ok);
                    wave_lds_sync();
                    // the weights are loaded where they are used (L1 hits), so
                    // that they do not hold registers across the features
                    const MlpLane L = mlp_lane(a.mlp, lane);
                    ph[m] = mlp_phi(mlp_rows_z(L, X, lane), ok);
                    wave_lds_sync();  // the rows are rewritten for the next edge
                    if (active) a.phi[3 * c + m] = ph[m];
                }
            } else if (active) {
#pragma unroll
                for (int m = 0; m < 3; ++m) ph[m] = ldx(a.phi, 3 * c + m);
            }
            T4 Uc{}, Un0{}, Un1{}, Un2{}, co0{}, co1{}, co2{};
            if (active) {
                Uc = ldx(a.Uin, c);
                Un0 = ldx(a.Uin, hn0 ? nb4.x : c);
                Un1 = ldx(a.Uin, hn1 ? nb4.y : c);
                Un2 = ldx(a.Uin, hn2 ? nb4.z : c);
                co0 = ldx(a.he_co, c);
                co1 = ldx(a.he_co, a.n + c);
                co2 = ldx(a.he_co, 2 * a.n + c);
            }
            if (active) {
                Ukeep = Uc;
                const unsigned word = (unsigned)nb4.w;
                sW[cl] = word;
                const Prim<T> pc = prim(Uc, eps);
                // a missing neighbour's slot holds the cell's own state
                const Prim<T> pn[3] = {prim(Un0, eps), prim(Un1, eps), prim(Un2, eps)};
                const bool hn[3] = {hn0, hn1, hn2};
                const int nb[3] = {nb4.x, nb4.y, nb4.z};
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const int k = nb[m];
                    sK[m * TILE + cl] = k;
                    const unsigned jb = (word >> (2 * m)) & 3u, isL = (word >> (6 + m)) & 1u;
                    const unsigned ent = (unsigned)m | ((unsigned)cl << 2) | (jb << 12) | (isL << 14);
                    if (k < 0) {  // boundary half-edge: a task of its own
                        sTask[atomicAdd(&sCount[0], 1)] = ent;
                        continue;
                    }
                    const T4 co = m == 0 ? co0 : (m == 1 ? co1 : co2);
                    const T ga = ldx(a.he_gam, m * a.n + c);
                    const int ma = (m + 1) % 3, mb = (m + 2) % 3;
                    const Half<T> r = recon3<T, MUSCL_, RL>(pc, pn[m], pn[ma], hn[ma], pn[mb], hn[mb],
                                                             co.x, co.y, co.z, co.w, ga, ph[m], eps);
                    T4 rv;
                    rv.x = r.h; rv.y = r.b; rv.z = r.un; rv.w = r.ut;
                    sR[m * TILE + cl] = rv;
                    sB[m * TILE + cl] = T(0.5) * g * (r.h + Uc.x) * (r.eta - (pc.h + pc.b));
                    const int kl = k - c0;
                    if (kl >= 0 && kl < TILE) {
                        if (isL) sTask[3 * TILE - 1 - atomicAdd(&sCount[1], 1)] = ent | ((unsigned)kl << 15);
                    } else {
                        sTask[atomicAdd(&sCount[0], 1)] = ent;
                    }
                }
            }
        } else if (active) {
            const T4 Uc = ldx(a.Uin, c);
            Ukeep = Uc;
            const int nb[3] = {nb4.x, nb4.y, nb4.z};
            const unsigned word = (unsigned)nb4.w;
            sW[cl] = word;
            const Prim<T> pc = prim(Uc, eps);
            Prim<T> pn[3];
            bool hn[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                hn[m] = nb[m] >= 0;
                pn[m] = hn[m] ? prim(a.Uin[nb[m]], eps) : pc;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const int k = nb[m];
                sK[m * TILE + cl] = k;
                const unsigned jb = (word >> (2 * m)) & 3u, isL = (word >> (6 + m)) & 1u;
                const unsigned ent = (unsigned)m | ((unsigned)cl << 2) | (jb << 12) | (isL << 14);
                if (k < 0) {  // boundary half-edge: a task of its own
                    sTask[atomicAdd(&sCount[0], 1)] = ent;
                    continue;
                }
                const T4 co = ldx(a.he_co, m * a.n + c);
                const int ma = (m + 1) % 3, mb = (m + 2) % 3;
                const Half<T> r = recon3<T, MUSCL_, LIM>(pc, pn[m], pn[ma], hn[ma], pn[mb], hn[mb],
                                                          co.x, co.y, co.z, co.w, T(0), 0.0f, eps);
                T4 rv;
                rv.x = r.h; rv.y = r.b; rv.z = r.un; rv.w = r.ut;
                sR[m * TILE + cl] = rv;
                // side correction and centred bed term less the cell's
                // hydrostatic pressure: g (h- + h)(eta- - eta) / 2 along n
                sB[m * TILE + cl] = T(0.5) * g * (r.h + Uc.x) * (r.eta - (pc.h + pc.b));
                const int kl = k - c0;
                if (kl >= 0 && kl < TILE) {
                    if (isL) sTask[3 * TILE - 1 - atomicAdd(&sCount[1], 1)] = ent | ((unsigned)kl << 15);
                } else {
                    sTask[atomicAdd(&sCount[0], 1)] = ent;
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        // ---- 2: edge tasks, one dense sweep (outside-tile edges first)
        {
            const int n0 = sCount[0], nt = n0 + sCount[1];
            // learned limiter: every thread runs the same number of sweeps,
            // so that a wave evaluates the network as a whole
            const int iend = kNet ? (nt + TILE - 1) / TILE * TILE : nt;
            for (int i = threadIdx.x; i < iend; i += TILE) {
                float phin = 0.0f;  // learned, first stage: phi of an outside edge's far side
                if constexpr (kNet) {
                    if (i - (int)threadIdx.x < n0) {
                        // the far side's own half-edge, from its 1-ring of U^n
                        // (the tile that owns it evaluates the same bits)
                        T4 Uk{}, Ut{}, Ua{}, Ub{}, ck{};
                        bool hk = false, ha = false, hb = false;
                        if (i < n0) {
                            const unsigned task = sTask[i];
                            const int m = task & 3u, tl = (task >> 2) & 1023u, jb = (task >> 12) & 3u;
                            const int k = sK[m * TILE + tl];
                            if (k >= 0) {
                                const int4 nk = ldx(a.nbr, k);
                                const int ka = pick3(nk, (jb + 1) % 3), kb = pick3(nk, (jb + 2) % 3);
                                hk = true;
                                ha = ka >= 0;
                                hb = kb >= 0;
                                Uk = ldx(a.Uin, k);
                                Ut = ldx(a.Uin, c0 + tl);
                                Ua = ldx(a.Uin, ha ? ka : k);
                                Ub = ldx(a.Uin, hb ? kb : k);
                                ck = ldx(a.he_co, jb * a.n + k);
                            }
                        }
                        float f[kMlpIn];
                        const bool ok = limiter_features<T, T4>(Uk, Ut, hk, Ua, ha, Ub, hb, ck.x, ck.y,
                                                                ck.z, ck.w, g, eps, f);
                        const int lane = threadIdx.x & 63;
                        uint16_t(*X)[16] = sX + (threadIdx.x & ~63);
                        const MlpLane L = mlp_lane(a.mlp, lane);
                        mlp_write_row(X[lane], f, ok);
                        wave_lds_sync();
                        phin = mlp_phi(mlp_rows_z(L, X, lane), ok);
                        wave_lds_sync();
                    }
                    if (i >= nt) continue;
                }
                const bool inside = i >= n0;
                const unsigned task = inside ? sTask[3 * TILE - 1 - (i - n0)] : sTask[i];
                const int m = task & 3u, tl = (task >> 2) & 1023u, jb = (task >> 12) & 3u;
                const bool isL = (task >> 14) & 1u;
                const int kl = inside ? (int)((task >> 15) & 1023u) : -1;
                const int tc = c0 + tl;
                const int k = inside ? c0 + kl : sK[m * TILE + tl];
                const T4 co = ldx(a.he_co, m * a.n + tc);
                const T nx = co.x, ny = co.y;
                if (k < 0) {  // boundary flux (Sec. 6.1), in the global frame
                    const T4 Ut = ldx(a.Uin, tc);
                    const int st = (int)(sW[tl] >> kScenShift);
                    const ScenParams sp = a.scen[st];
                    T q_in = T(0);
                    if (k == kBcInflow) {
                        const double t_st =
                            bitsd(a.clock[clock_off(a.ncopy, st, a.slot_cur)]) +
                            (a.kind == 2 ? lane_step_dt(a.clock, a.ncopy, a.slot_cur, st, a.cfl_rule,
                                                        a.cfl, a.dt_max, a.dt_fixed)
                                         : 0.0);
                        q_in = T(inflow_at(sp, a.ser_t, a.ser_q, t_st) * sp.inv_inflow_len);
                    }
                    T G[3];
                    boundary_flux_dev<T, T4>(k, Ut, nx, ny, g, eps, q_in, T(sp.outflow_stage), G);
                    T4 fb;
                    fb.x = G[0]; fb.y = G[1]; fb.z = G[2]; fb.w = T(0);
                    sR[m * TILE + tl] = fb;
                    continue;
                }
                const T4 ov = sR[m * TILE + tl];
                const T sbo = sB[m * TILE + tl];
                T4 kv;
                T sbk = T(0);
                if (inside) {
                    kv = sR[jb * TILE + kl];
                    sbk = sB[jb * TILE + kl];
                } else {
                    // far side: its own reconstruction across this edge, from its 2-ring
                    const Prim<T> pk = prim(ldx(a.Uin, k), eps);
                    const Prim<T> pc = prim(ldx(a.Uin, tc), eps);
                    Prim<T> pka = pk, pkb = pk;
                    bool hka = false, hkb = false;
                    T al = T(0), be = T(0), ga = T(0);
                    float phik = 0.0f;
                    if (MUSCL_) {
                        const int4 nk = ldx(a.nbr, k);
                        const int ka = pick3(nk, (jb + 1) % 3), kb = pick3(nk, (jb + 2) % 3);
                        hka = ka >= 0;
                        hkb = kb >= 0;
                        if (hka) pka = prim(ldx(a.Uin, ka), eps);
                        if (hkb) pkb = prim(ldx(a.Uin, kb), eps);
                        const T4 ck = ldx(a.he_co, jb * a.n + k);
                        al = ck.z;
                        be = ck.w;
                        if (RL == kLearned) {
                            ga = ldx(a.he_gam, jb * a.n + k);
                            phik = kNet ? phin : ldx(a.phi, 3 * k + jb);
                        }
                    }
                    const Half<T> r = recon3<T, MUSCL_, RL>(pk, pc, pka, hka, pkb, hkb, -nx, -ny, al,
                                                              be, ga, phik, eps);
                    kv.x = r.h; kv.y = r.b; kv.z = r.un; kv.w = r.ut;
                }
                // hydrostatic reconstruction
                const T bmax = tmax(ov.y, kv.y);
                const T hso = tmax(T(0), ov.x + ov.y - bmax);
                const T hsk = tmax(T(0), kv.x + kv.y - bmax);
                // HLLC in the canonical orientation: operands selected, one
                // evaluation, whichever side files the edge
                const T hL = isL ? hso : hsk, uL = isL ? ov.z : kv.z, vL = isL ? ov.w : kv.w;
                const T hR = isL ? hsk : hso, uR = isL ? -kv.z : -ov.z, vR = isL ? -kv.w : -ov.w;
                const T nLx = isL ? nx : -nx, nLy = isL ? ny : -ny;
                T F0, DL, DR, F2;
                hllc_dev(g, eps, hL, uL, vL, hR, uR, vR, F0, DL, DR, F2);
                const T sg = isL ? T(1) : T(-1);
                // each side's normal momentum flux less its own hydrostatic
                // pressure, rotated back from the canonical frame
                const T Do = isL ? DL : DR;
                T4 fo;
                half_edge_flux(sg, F0, Do * nLx - F2 * nLy, Do * nLy + F2 * nLx, sbo, nx, ny, fo.x,
                               fo.y, fo.z);
                fo.w = T(0);
                sR[m * TILE + tl] = fo;
                if (inside) {  // the other cell's half-edge: normal -n, sign -sg
                    const T Dk = isL ? DR : DL;
                    T4 fk;
                    half_edge_flux(-sg, F0, Dk * nLx - F2 * nLy, Dk * nLy + F2 * nLx, sbk, -nx, -ny,
                                   fk.x, fk.y, fk.z);
                    fk.w = T(0);
                    sR[jb * TILE + kl] = fk;
                }
            }
        }
        __syncthreads();
        // the update ends the tile and frees its slot for the next one: above
        // the edge sweeps of other tiles, below their first phases
        __builtin_amdgcn_s_setprio(2);
        // ---- 3: cell sums, update, friction, cleanup, CFL
        CflVal<T> cfl = cfl_none<T>();
        const T4 Uc = Ukeep;
        const unsigned word = active ? sW[cl] : 0u;
        const int s = active ? (int)(word >> kScenShift) : -1;
        const double dtd = dt_finish(dtp, a.clock, a.ncopy, a.slot_cur, s, a.cfl_rule, a.cfl,
                                     a.dt_max, a.dt_fixed);
        if (active) {
            const T dt = T(dtd);
            T acc0 = T(0), acc1 = T(0), acc2 = T(0), lsum = T(0);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const T lam = ldx(a.he_lam, m * a.n + c);
                const T4 f = sR[m * TILE + cl];
                acc0 += lam * f.x;
                acc1 += lam * f.y;
                acc2 += lam * f.z;
                lsum += lam;
            }
            T nh = Uc.x - dt * acc0;
            T nu = Uc.y - dt * acc1;
            T nv = Uc.z - dt * acc2;
            // the inscribed radius from the edge weights: sum_m L_m / |Omega|
            // = P / |Omega|, so R = 2 |Omega| / P = 2 / that sum; Manning's
            // n^2 is the only per-cell value read (4 bytes, not 16)
            T4 cg;
            cg.y = fdiv(T(2), lsum);
            cg.z = ldx(a.man2, c);
            int flags = 0;
            if (!(isfinite(nh) && isfinite(nu) && isfinite(nv))) flags |= kHealthNonfinite;
            if (nh < T(0)) {
                flags |= nh < -eps ? kHealthNegDepth : kHealthClipped;
                nh = T(0);
            }
            if (nh <= eps) {
                nu = T(0); nv = T(0);
            } else if (cg.z > T(0)) {  // Manning, point-implicit
                const T sp = sqrt(nu * nu + nv * nv) * frcp(nh);
                const T f = T(1) + dt * g * cg.z * sp * pow_m43(nh);
                const T rf = frcp(f);
                nu *= rf; nv *= rf;
            }
            if (a.kind == 2) {
                const T4 U0c = ldx(a.U0, c);
                nh = T(0.5) * (U0c.x + nh);
                nu = T(0.5) * (U0c.y + nu);
                nv = T(0.5) * (U0c.z + nv);
                if (nh <= eps) { nu = T(0); nv = T(0); }
            }
            T4 out;
            out.x = nh; out.y = nu; out.z = nv; out.w = Uc.w;
            stx(a.Uout, c, out);
            pack_own(a, c, nh, nu, nv);
            // health counts owned cells: a ghost cell's new state is provisional
            // (the next exchange replaces it)
            if (flags && ((word >> kOwnedBit) & 1u)) atomicOr(a.health, flags);
            cfl.scen = s;
            if (a.kind != 1 && ((word >> kOwnedBit) & 1u) && nh > eps) {
                const T r = frcp(nh);
                const T u = nu * r, v = nv * r;
                const T lm = sqrt(u * u + v * v) + sqrt(g * nh);
                cfl = cfl_cell<T>(a.cfl_rule, s, cg.y, lm);
            }
        }
        if (a.kind != 1) cfl_commit(a.clock, a.ncopy, a.slot_next, a.cfl_rule, cfl, sCfl);
        __builtin_amdgcn_s_setprio(0);
        if (tile + (int)gridDim.x < ntiles) __syncthreads();  // LDS is reused by the next tile
    }
}

// Tiled WAF stage (Euler).  The tiling of k_stage_tiled with WAF's data:
//  1. every thread stores, per interior half-edge of its cell, the
//     first-order interface values (h, b, u_n, u_t in its own edge frame),
//     the cell's eta and tangential velocity and the mean eta and
//     tangential velocity of its two upwind cells (WAF's ratios,
//     Sec. 6.2.2), and files the edge tasks as k_stage_tiled does; the
//     cell's step goes to LDS too (the Courant numbers need it);
//  2. one dense sweep over the tasks: hydrostatic reconstruction, WAF in the
//     canonical orientation (operands selected, one evaluation; an edge
//     leaving the tile recomputes the far side from its 2-ring), rotation
//     back, each side's share with its side correction (printed form);
//  3. cell sums, update, Manning, cleanup, CFL commit.
// Tangential velocities taken in a cell's own frame are negated when that
// frame is opposite to the canonical one (exact), so an edge gets the same
// operands, and the same flux bits, wherever it is evaluated.
template <typename T, int WAFM, int TILE>
__global__ void __launch_bounds__(TILE) k_stage_tiled_waf(StageArgs<T> a)
{
    using T4 = typename V4<T>::type;
    static_assert(TILE <= 1024, "10-bit tile-local indices in task entries");
    __shared__ T4 sR[3 * TILE];        // own-frame h, b, u_n, u_t
    __shared__ T4 sQ[3 * TILE];        // eta, u_t (tangential form) of the cell; same of its upwind mean
    __shared__ unsigned char sH[3 * TILE];  // the half-edge has an upwind cell
    __shared__ unsigned sTask[3 * TILE];
    __shared__ int sK[3 * TILE];
    __shared__ T sRad[TILE];           // inscribed radius of each cell (positivity)
    __shared__ T sDt[TILE];
    __shared__ int sCount[2];
    __shared__ CflVal<T> sCfl[TILE / 64];
    clock_upkeep(a);
    const T g = a.g, eps = a.eps;
    const int ntiles = (a.n + TILE - 1) / TILE;
    for (int tile = xcd_tile(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
        const int c0 = tile * TILE, cl = threadIdx.x, c = c0 + cl;
        const bool active = c < a.n;
        if (threadIdx.x < 2) sCount[threadIdx.x] = 0;
        __syncthreads();
        // ---- 1
        int4 nb4 = make_int4(-1, -1, -1, 0);
        if (active) nb4 = ldx(a.nbr, c);
        const DtPrefetch dtp = dt_prefetch(a.clock, a.ncopy, a.slot_cur,
                                           active ? (int)((unsigned)nb4.w >> kScenShift) : -1, a.dt_fixed);
        T4 Ukeep;
        T man2 = T(0);
        const unsigned word = (unsigned)nb4.w;
        if (active) {
            const T4 Uc = ldx(a.Uin, c);
            Ukeep = Uc;
            const T4 cg = ldx(a.cell, c);
            sRad[cl] = cg.y;
            man2 = cg.z;
            const bool hn0 = nb4.x >= 0, hn1 = nb4.y >= 0, hn2 = nb4.z >= 0;
            const T4 Un0 = a.Uin[hn0 ? nb4.x : c], Un1 = a.Uin[hn1 ? nb4.y : c], Un2 = a.Uin[hn2 ? nb4.z : c];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const int k = m == 0 ? nb4.x : (m == 1 ? nb4.y : nb4.z);
                sK[m * TILE + cl] = k;
                const unsigned jb = (word >> (2 * m)) & 3u, isL = (word >> (6 + m)) & 1u;
                const unsigned ent = (unsigned)m | ((unsigned)cl << 2) | (jb << 12) | (isL << 14);
                if (k < 0) {
                    sTask[atomicAdd(&sCount[0], 1)] = ent;
                    continue;
                }
                const int ma = (m + 1) % 3, mb = (m + 2) % 3;
                const T4 Ua = ma == 0 ? Un0 : (ma == 1 ? Un1 : Un2);
                const T4 Ub = mb == 0 ? Un0 : (mb == 1 ? Un1 : Un2);
                const bool ha = ma == 0 ? hn0 : (ma == 1 ? hn1 : hn2);
                const bool hb = mb == 0 ? hn0 : (mb == 1 ? hn1 : hn2);
                const auto ge = ldx(a.he_nrm, m * a.n + c);  // unit normal
                T4 rv;
                rv.x = Uc.x;
                rv.y = Uc.w;
                frame_vel(Uc, ge.x, ge.y, eps, rv.z, rv.w);
                sR[m * TILE + cl] = rv;
                T eu, vu;
                const bool hu = waf_upwind(Ua, ha, Ub, hb, ge.x, ge.y, eps, eu, vu);
                T4 q;
                q.x = Uc.x + Uc.w;
                q.y = tangential(Uc, ge.x, ge.y, eps);
                q.z = eu;
                q.w = vu;
                sQ[m * TILE + cl] = q;
                sH[m * TILE + cl] = hu ? 1 : 0;
                const int kl = k - c0;
                if (kl >= 0 && kl < TILE) {
                    if (isL) sTask[3 * TILE - 1 - atomicAdd(&sCount[1], 1)] = ent | ((unsigned)kl << 15);
                } else {
                    sTask[atomicAdd(&sCount[0], 1)] = ent;
                }
            }
        }
        const int s = active ? (int)(word >> kScenShift) : -1;
        const double dtd = dt_finish(dtp, a.clock, a.ncopy, a.slot_cur, s, a.cfl_rule, a.cfl,
                                     a.dt_max, a.dt_fixed);
        sDt[cl] = T(dtd);
        __syncthreads();
        // ---- 2
        {
            const int n0 = sCount[0], nt = n0 + sCount[1];
            for (int i = threadIdx.x; i < nt; i += TILE) {
                const bool inside = i >= n0;
                const unsigned task = inside ? sTask[3 * TILE - 1 - (i - n0)] : sTask[i];
                const int m = task & 3u, tl = (task >> 2) & 1023u, jb = (task >> 12) & 3u;
                const bool isL = (task >> 14) & 1u;
                const int kl = inside ? (int)((task >> 15) & 1023u) : -1;
                const int tc = c0 + tl;
                const int k = inside ? c0 + kl : sK[m * TILE + tl];
                const auto ge = ldx(a.he_nrm, m * a.n + tc);
                const T nx = ge.x, ny = ge.y;
                if (k < 0) {  // boundary flux (Sec. 6.1), printed form, global frame
                    const T4 Ut = ldx(a.Uin, tc);
                    const int st = (int)((unsigned)ldx(a.nbr, tc).w >> kScenShift);
                    const ScenParams sp = a.scen[st];
                    const T q_in = k == kBcInflow
                                       ? T(inflow_at(sp, a.ser_t, a.ser_q,
                                                     bitsd(a.clock[clock_off(a.ncopy, st, a.slot_cur)])) *
                                           sp.inv_inflow_len)
                                       : T(0);
                    T G[3];
                    boundary_flux<T, T4>(k, Ut, nx, ny, g, eps, q_in, T(sp.outflow_stage), G);
                    T4 fb;
                    fb.x = G[0]; fb.y = G[1]; fb.z = G[2]; fb.w = T(0);
                    sR[m * TILE + tl] = fb;
                    continue;
                }
                const T4 ov = sR[m * TILE + tl], oq = sQ[m * TILE + tl];
                const bool oh = sH[m * TILE + tl] != 0;
                T4 kv, kq;
                bool kh;
                if (inside) {
                    kv = sR[jb * TILE + kl];
                    kq = sQ[jb * TILE + kl];
                    kh = sH[jb * TILE + kl] != 0;
                } else {
                    // far side from its 2-ring, in its own frame (normal -n)
                    const T4 Uk = ldx(a.Uin, k);
                    const int4 nk = ldx(a.nbr, k);
                    const int ka = pick3(nk, (jb + 1) % 3), kb = pick3(nk, (jb + 2) % 3);
                    const T4 Uka = a.Uin[ka >= 0 ? ka : k], Ukb = a.Uin[kb >= 0 ? kb : k];
                    kv.x = Uk.x;
                    kv.y = Uk.w;
                    frame_vel(Uk, -nx, -ny, eps, kv.z, kv.w);
                    T eu, vu;
                    kh = waf_upwind(Uka, ka >= 0, Ukb, kb >= 0, -nx, -ny, eps, eu, vu);
                    kq.x = Uk.x + Uk.w;
                    kq.y = tangential(Uk, -nx, -ny, eps);
                    kq.z = eu;
                    kq.w = vu;
                }
                // hydrostatic reconstruction (first-order states)
                const T be = tmax(ov.y, kv.y);
                const T hso = tmax(T(0), ov.x + ov.y - be);
                const T hsk = tmax(T(0), kv.x + kv.y - be);
                // canonical orientation: L's own frame is the canonical one,
                // R's is opposite (its normal and tangential components flip)
                const T4 &Lv = isL ? ov : kv, &Rv = isL ? kv : ov, &Lq = isL ? oq : kq, &Rq = isL ? kq : oq;
                const T hL = isL ? hso : hsk, hR = isL ? hsk : hso;
                T UL[3], UR[3];
                UL[0] = hL; UL[1] = hL * Lv.z; UL[2] = hL * Lv.w;
                UR[0] = hR; UR[1] = -(hR * Rv.z); UR[2] = -(hR * Rv.w);
                WafIn<T> w;
                w.eL = Lq.x; w.eR = Rq.x;
                w.vL = Lq.y; w.vR = -Rq.y;
                w.eLu = Lq.z; w.eRu = Rq.z;
                w.vLu = Lq.w; w.vRu = -Rq.w;
                w.hasLu = isL ? oh : kh;
                w.hasRu = isL ? kh : oh;
                T F[3];
                const T dtt = sDt[tl];
                flux_waf<T, WAFM>(g, eps, fdiv(dtt, ldx(a.he_dfw, m * a.n + tc)), UL, UR, w, F);
                if (a.waf_pos) {
                    const T Ro = sRad[tl];
                    const T Rk = inside ? sRad[kl] : ((const T *)a.cell)[4 * (size_t)k + 1];
                    waf_positivity(g, eps, UL, UR, Lv.x, isL ? Ro : Rk, Rv.x, isL ? Rk : Ro, dtt, F);
                }
                const T sg = isL ? T(1) : T(-1);
                const T nLx = sg * nx, nLy = sg * ny;
                const T G0 = F[0], G1 = F[1] * nLx - F[2] * nLy, G2 = F[1] * nLy + F[2] * nLx;
                T4 fo;
                half_edge_flux(sg, G0, G1, G2, T(0.5) * g * (ov.x * ov.x - hso * hso), nx, ny, fo.x,
                               fo.y, fo.z);
                fo.w = T(0);
                sR[m * TILE + tl] = fo;
                if (inside) {
                    T4 fk;
                    half_edge_flux(-sg, G0, G1, G2, T(0.5) * g * (kv.x * kv.x - hsk * hsk), -nx, -ny,
                                   fk.x, fk.y, fk.z);
                    fk.w = T(0);
                    sR[jb * TILE + kl] = fk;
                }
            }
        }
        __syncthreads();
        // ---- 3
        CflVal<T> cfl = cfl_none<T>();
        if (active) {
            const T4 Uc = Ukeep;
            const T dt = sDt[cl];
            T acc0 = T(0), acc1 = T(0), acc2 = T(0);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const T lam = ldx(a.he_lam, m * a.n + c);
                const T4 f = sR[m * TILE + cl];
                acc0 += lam * f.x;
                acc1 += lam * f.y;
                acc2 += lam * f.z;
            }
            T nh = Uc.x - dt * acc0;
            T nu = Uc.y - dt * acc1;
            T nv = Uc.z - dt * acc2;
            int flags = 0;
            if (!(isfinite(nh) && isfinite(nu) && isfinite(nv))) flags |= kHealthNonfinite;
            if (nh < T(0)) {
                flags |= nh < -eps ? kHealthNegDepth : kHealthClipped;
                nh = T(0);
            }
            if (nh <= eps) {
                nu = T(0); nv = T(0);
            } else if (man2 > T(0)) {  // Manning, point-implicit
                const T sp = sqrt(nu * nu + nv * nv) * frcp(nh);
                const T f = T(1) + dt * g * man2 * sp * pow_m43(nh);
                const T rf = frcp(f);
                nu *= rf; nv *= rf;
            }
            T4 out;
            out.x = nh; out.y = nu; out.z = nv; out.w = Uc.w;
            stx(a.Uout, c, out);
            pack_own(a, c, nh, nu, nv);
            // health counts owned cells: a ghost cell's new state is provisional
            // (the next exchange replaces it)
            if (flags && ((word >> kOwnedBit) & 1u)) atomicOr(a.health, flags);
            cfl.scen = s;
            if (((word >> kOwnedBit) & 1u) && nh > eps) {
                const T r = frcp(nh);
                const T u = nu * r, v = nv * r;
                const T lm = sqrt(u * u + v * v) + sqrt(g * nh);
                cfl = cfl_cell<T>(a.cfl_rule, s, sRad[cl], lm);
            }
        }
        cfl_commit(a.clock, a.ncopy, a.slot_next, a.cfl_rule, cfl, sCfl);
        if (tile + (int)gridDim.x < ntiles) __syncthreads();
    }
}

// CFL minima of the current state into one clock slot (after set_state).
template <typename T>
__global__ void __launch_bounds__(256) k_cfl_init(int n, const int4 *nbr,
                                                  const typename V4<T>::type *cell,
                                                  const typename V4<T>::type *U, ClockWord *clock,
                                                  int ncopy, int slot, int rule, T g, T eps)
{
    __shared__ CflVal<T> part[4];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    CflVal<T> v = cfl_none<T>();
    if (c < n) {
        const unsigned word = (unsigned)nbr[c].w;
        const T h = U[c].x;
        if (((word >> kOwnedBit) & 1u) && h > eps) {
            const T u = fdiv(U[c].y, h), w = fdiv(U[c].z, h);
            const T lm = sqrt(u * u + w * w) + sqrt(g * h);
            v = cfl_cell<T>(rule, (int)(word >> kScenShift), cell[c].y, lm);
        }
        v.scen = (int)(word >> kScenShift);
    }
    cfl_commit(clock, ncopy, slot, rule, v, part);
}

// Clock slot `slot` of every scenario: partials cleared, time set from t0
// when set_t.  One thread per (scenario, copy).
__global__ void k_clock_reset(ClockWord *clock, int ncopy, int n_scen, int slot, const double *t0,
                              int set_t)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_scen * ncopy) return;
    const int s = e / ncopy, j = e % ncopy;
    ClockWord *q = clock + clock_off(ncopy, s, slot);
    if (set_t && j == 0) q[0] = dbits(t0[s]);
    q += (size_t)(1 + j) * kClockLine;
    q[kCfqMin] = kInfBits;
    q[kCfqMax] = 0ull;
}

template <typename T>
__global__ void k_pack_state(int n, const T *h, const T *hu, const T *hv, const T *b,
                             typename V4<T>::type *U, int *bad, T eps)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    typename V4<T>::type u;
    u.x = h[c]; u.y = hu[c]; u.z = hv[c]; u.w = b[c];
    if (!(isfinite(u.x) && isfinite(u.y) && isfinite(u.z)) || u.x < T(0)) atomicOr(bad, 1);
    U[c] = u;
}

template <typename T>
__global__ void k_unpack_state(int n, const typename V4<T>::type *U, T *h, T *hu, T *hv)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const typename V4<T>::type u = U[c];
    h[c] = u.x; hu[c] = u.y; hv[c] = u.z;
}

// Send buffer [3][n_send] from the owned cells listed in send_idx (Sec. 6.4).
template <typename T>
__global__ void k_pack_ghosts(int n_send, const int *send_idx, const typename V4<T>::type *U,
                              T *buf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_send) return;
    const typename V4<T>::type u = U[send_idx[i]];
    buf[i] = u.x;
    buf[n_send + i] = u.y;
    buf[2 * n_send + i] = u.z;
}

// In-place receive: [3][n_ghost] into the contiguous ghost range.
template <typename T>
__global__ void k_unpack_ghosts(int n_owned, int n_ghost, const T *buf, typename V4<T>::type *U)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ghost) return;
    typename V4<T>::type u = U[n_owned + i];
    u.x = buf[i]; u.y = buf[n_ghost + i]; u.z = buf[2 * n_ghost + i];
    U[n_owned + i] = u;
}

__global__ void k_fill_int(int *p, int v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

namespace {

constexpr int kGraphSteps = 6;  // lcm of the clock-slot (3) and buffer (2) periods

int set_err(swe_ctx *c, int code, const std::string &m)
{
    if (c) c->err = m;
    return code;
}

#define HIP_OK(ctx, expr)                                                                 \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return set_err(ctx, e_ == hipErrorOutOfMemory ? SWE_ERR_OOM : SWE_ERR_DEVICE, \
                           std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

template <typename P> void dfree_t(swe_ctx *c, P *&p)
{
    void *v = p;
    dfree(c, v);
    p = nullptr;
}

void release_mesh(swe_ctx *c)
{
    if (c->graph) { (void)hipGraphExecDestroy(c->graph); c->graph = nullptr; }
    dfree(c, c->nbr); dfree(c, c->cell); dfree(c, c->man2); dfree(c, c->he_geo); dfree(c, c->he_dist);
    dfree(c, c->he_co); dfree(c, c->he_lam); dfree(c, c->he_gam); dfree(c, c->he_dfw); dfree(c, c->he_nrm);
    dfree(c, c->U[0]); dfree(c, c->U[1]); dfree(c, c->U1); dfree(c, c->tmp3); dfree(c, c->bed);
    dfree_t(c, c->phi); dfree_t(c, c->clock); dfree_t(c, c->scen); dfree_t(c, c->ser_t); dfree_t(c, c->ser_q);
    dfree_t(c, c->t0); dfree_t(c, c->send_idx); dfree_t(c, c->pk_off); dfree_t(c, c->pk_ent);
    c->has_mesh = c->has_state = false;
}

size_t clock_bytes(const swe_ctx *c)
{
    return sizeof(ClockWord) * clock_off(c->ncopy, c->n_scen, 0);
}

template <typename T>
void to_t(const std::vector<double> &src, std::vector<T> &dst)
{
    dst.resize(src.size());
    for (size_t i = 0; i < src.size(); ++i) dst[i] = T(src[i]);
}

template <typename T>
int upload_geometry(swe_ctx *c, const HostGeometry &g)
{
    const size_t n = c->n_total;
    std::vector<T> tmp;
    HIP_OK(c, dalloc(c, (void **)&c->nbr, 16 * n));
    HIP_OK(c, hipMemcpy(c->nbr, g.nbr4.data(), 16 * n, hipMemcpyHostToDevice));
    to_t(g.cell, tmp);
    HIP_OK(c, dalloc(c, (void **)&c->cell, 4 * sizeof(T) * n));
    HIP_OK(c, hipMemcpy(c->cell, tmp.data(), 4 * sizeof(T) * n, hipMemcpyHostToDevice));
    {
        std::vector<T> m2(n);
        for (size_t i = 0; i < n; ++i) m2[i] = tmp[4 * i + 2];
        HIP_OK(c, dalloc(c, (void **)&c->man2, sizeof(T) * n));
        HIP_OK(c, hipMemcpy(c->man2, m2.data(), sizeof(T) * n, hipMemcpyHostToDevice));
    }
    to_t(g.he_geo, tmp);
    HIP_OK(c, dalloc(c, (void **)&c->he_geo, 12 * sizeof(T) * n));
    HIP_OK(c, hipMemcpy(c->he_geo, tmp.data(), 12 * sizeof(T) * n, hipMemcpyHostToDevice));
    to_t(g.he_dist, tmp);
    HIP_OK(c, dalloc(c, (void **)&c->he_dist, 12 * sizeof(T) * n));
    HIP_OK(c, hipMemcpy(c->he_dist, tmp.data(), 12 * sizeof(T) * n, hipMemcpyHostToDevice));
    // compact half-edge set of the tiled kernel, formed in double and
    // rounded once: unit normal, the two MUSCL slope weights (the limiters
    // are positively homogeneous of degree one, so d_mid * lim(sb, sf) =
    // lim(d_mid sb, d_mid sf)), the learned limiter's central weight and the
    // edge length over the cell area
    // Stored edge-major (half-edge m of cell c at m * n + c), so that a
    // wave's loads of one local edge are contiguous.
    // The tiled WAF kernel takes the unit normal and the centroid distance
    // of its Courant numbers from two more edge-major arrays (WAF contexts
    // only): it has no use for the MUSCL weights.
    const bool waf = c->cfg.scheme == SWE_WAF;
    std::vector<T> co(12 * n), lam(3 * n), gam(3 * n), dfw(waf ? 3 * n : 0), nrm(waf ? 6 * n : 0);
    for (size_t cc = 0; cc < n; ++cc)
        for (size_t m = 0; m < 3; ++m) {
            const size_t h = 3 * cc + m, e = m * n + cc;
            const double *ge = &g.he_geo[4 * h], *gd = &g.he_dist[4 * h];
            co[4 * e + 0] = T(ge[0]);
            co[4 * e + 1] = T(ge[1]);
            co[4 * e + 2] = T(ge[3] * gd[0]);
            co[4 * e + 3] = T(ge[3] * gd[1]);
            lam[e] = T(ge[2] * g.cell[4 * cc]);
            gam[e] = T(ge[3] * gd[2]);
            if (waf) {
                dfw[e] = T(gd[3]);
                nrm[2 * e] = T(ge[0]);
                nrm[2 * e + 1] = T(ge[1]);
            }
        }
    if (waf) {
        HIP_OK(c, dalloc(c, (void **)&c->he_dfw, 3 * sizeof(T) * n));
        HIP_OK(c, hipMemcpy(c->he_dfw, dfw.data(), 3 * sizeof(T) * n, hipMemcpyHostToDevice));
        HIP_OK(c, dalloc(c, (void **)&c->he_nrm, 6 * sizeof(T) * n));
        HIP_OK(c, hipMemcpy(c->he_nrm, nrm.data(), 6 * sizeof(T) * n, hipMemcpyHostToDevice));
    }
    HIP_OK(c, dalloc(c, (void **)&c->he_co, 12 * sizeof(T) * n));
    HIP_OK(c, hipMemcpy(c->he_co, co.data(), 12 * sizeof(T) * n, hipMemcpyHostToDevice));
    HIP_OK(c, dalloc(c, (void **)&c->he_lam, 3 * sizeof(T) * n));
    HIP_OK(c, hipMemcpy(c->he_lam, lam.data(), 3 * sizeof(T) * n, hipMemcpyHostToDevice));
    HIP_OK(c, dalloc(c, (void **)&c->he_gam, 3 * sizeof(T) * n));
    HIP_OK(c, hipMemcpy(c->he_gam, gam.data(), 3 * sizeof(T) * n, hipMemcpyHostToDevice));
    return SWE_OK;
}

int push_scenarios(swe_ctx *c)
{
    // the buffers below are replaced: the stream must be done with them
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->h_ser_t.clear();
    c->h_ser_q.clear();
    for (size_t i = 0; i < c->h_scen.size(); ++i) {
        c->h_scen[i].series_off = (int)c->h_ser_t.size();
        c->h_scen[i].series_n = i < c->series.size() ? (int)c->series[i].first.size() : 0;
        if (i < c->series.size()) {
            c->h_ser_t.insert(c->h_ser_t.end(), c->series[i].first.begin(), c->series[i].first.end());
            c->h_ser_q.insert(c->h_ser_q.end(), c->series[i].second.begin(), c->series[i].second.end());
        }
    }
    dfree_t(c, c->scen); dfree_t(c, c->ser_t); dfree_t(c, c->ser_q);
    HIP_OK(c, dalloc(c, (void **)&c->scen, sizeof(ScenParams) * c->h_scen.size()));
    HIP_OK(c, hipMemcpy(c->scen, c->h_scen.data(), sizeof(ScenParams) * c->h_scen.size(),
                        hipMemcpyHostToDevice));
    const size_t ns = std::max<size_t>(1, c->h_ser_t.size());
    HIP_OK(c, dalloc(c, (void **)&c->ser_t, sizeof(double) * ns));
    HIP_OK(c, dalloc(c, (void **)&c->ser_q, sizeof(double) * ns));
    if (!c->h_ser_t.empty()) {
        HIP_OK(c, hipMemcpy(c->ser_t, c->h_ser_t.data(), sizeof(double) * c->h_ser_t.size(),
                            hipMemcpyHostToDevice));
        HIP_OK(c, hipMemcpy(c->ser_q, c->h_ser_q.data(), sizeof(double) * c->h_ser_q.size(),
                            hipMemcpyHostToDevice));
    }
    return SWE_OK;
}

template <typename T> using KernelFn = void (*)(StageArgs<T>);

template <typename T, int TILE, int OCC = SWE_TILED_WAVES> KernelFn<T> pick_tiled(int scheme, int lim)
{
    if (scheme == kHLLC1) return k_stage_tiled<T, false, kMinmod, TILE, OCC>;
    switch (lim) {
    case kSuperbee: return k_stage_tiled<T, true, kSuperbee, TILE, OCC>;
    case kVanAlbada: return k_stage_tiled<T, true, kVanAlbada, TILE, OCC>;
    case kLearned: return k_stage_tiled<T, true, kLearned, TILE>;
    case kLearnedNet: return k_stage_tiled<T, true, kLearnedNet, TILE>;
    case kZeroSlope: return k_stage_tiled<T, true, kZeroSlope, TILE, OCC>;
    default: return k_stage_tiled<T, true, kMinmod, TILE, OCC>;
    }
}

// Seven waves per SIMD instead of six for the FP32 tiled kernel with
// 256-cell tiles: each tile takes longer (72 registers instead of 80), but
// the chip holds 7 instead of 6 tiles per compute unit.  Worth it when that
// saves a round of tiles in a launch of at most two rounds (a sub-domain of
// about 400k cells: one round instead of two), and on a launch of many
// rounds (8 or more), which then runs as a persistent grid of 7 blocks per
// compute unit (measured 6% faster on the 13M-cell river); on
// config-2-sized meshes (a few rounds) six is faster.
template <typename T> bool seven_waves(const swe_ctx *c, int B)
{
    if (sizeof(T) != 4 || B != 256 || c->cfg.scheme == SWE_WAF || c->cfg.cell_kernel ||
        (c->cfg.scheme == SWE_MUSCL && c->cfg.limiter == SWE_LEARNED))
        return false;
    if (c->waves) return c->waves == 7;
    const long long nt = (c->n_total + B - 1) / B, s6 = 6LL * c->ncu, s7 = 7LL * c->ncu;
    if (s6 <= 0) return false;
    const long long r6 = (nt + s6 - 1) / s6, r7 = (nt + s7 - 1) / s7;
    if (r6 >= 8 && c->grid_persist >= 0) return true;  // persistent grid (see stage_grid)
    return r7 < r6 && r6 <= 2;
}

template <typename T> KernelFn<T> pick_cell_kernel(int scheme, int lim, int wafm);

// Stage kernel of a configuration: the tiled kernel for first-order HLLC and
// MUSCL (tile = block size 64, 128 or 256), the cell kernel for WAF.
template <typename T, int TILE> KernelFn<T> pick_tiled_waf(int wafm)
{
    if (wafm == kWafGodunov) return k_stage_tiled_waf<T, kWafGodunov, TILE>;
    if (wafm == kWafUnlimited) return k_stage_tiled_waf<T, kWafUnlimited, TILE>;
    return k_stage_tiled_waf<T, kWafSuperbee, TILE>;
}

template <typename T> KernelFn<T> pick_kernel(int scheme, int lim, int wafm, int block, int cell,
                                              bool w7, bool euler)
{
    if (scheme == kWAF && !cell && euler) {  // tiled WAF: Euler only (as the paper's WAF)
        if (block == 64) return pick_tiled_waf<T, 64>(wafm);
        if (block == 128 || sizeof(T) == 8) return pick_tiled_waf<T, 128>(wafm);
        return pick_tiled_waf<T, 256>(wafm);
    }
    if (scheme != kWAF && !cell) {
        if (block == 64) return pick_tiled<T, 64>(scheme, lim);
        if (block == 128) return pick_tiled<T, 128>(scheme, lim);
        if (block == 512 && sizeof(T) == 4) return pick_tiled<T, 512>(scheme, lim);
        if (w7 && sizeof(T) == 4) return pick_tiled<T, 256, 7>(scheme, lim);
        return pick_tiled<T, 256>(scheme, lim);
    }
    return pick_cell_kernel<T>(scheme, lim, wafm);
}

template <typename T> KernelFn<T> pick_cell_kernel(int scheme, int lim, int wafm)
{
    if (scheme == kHLLC1) return k_stage<T, kHLLC1, kMinmod, 0>;
    if (scheme == kWAF) {
        if (wafm == kWafGodunov) return k_stage<T, kWAF, kMinmod, kWafGodunov>;
        if (wafm == kWafUnlimited) return k_stage<T, kWAF, kMinmod, kWafUnlimited>;
        return k_stage<T, kWAF, kMinmod, kWafSuperbee>;
    }
    switch (lim) {
    case kSuperbee: return k_stage<T, kMUSCL, kSuperbee, 0>;
    case kVanAlbada: return k_stage<T, kMUSCL, kVanAlbada, 0>;
    case kLearned: return k_stage<T, kMUSCL, kLearned, 0>;
    case kZeroSlope: return k_stage<T, kMUSCL, kZeroSlope, 0>;
    default: return k_stage<T, kMUSCL, kMinmod, 0>;
    }
}

// Blocks of `kernel` (block size B) the whole chip holds at once (0 if the
// occupancy query fails).
inline int resident_blocks(const swe_ctx *c, const void *kernel, int B)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, B, 0) != hipSuccess) return 0;
    return per_cu * c->ncu;
}

// Blocks of a tiled stage launch: one per tile, or, when the configuration
// asks for it or the launch spans many rounds of tiles (8 or more), a
// persistent grid of the blocks the chip holds at once, each sweeping tiles
// (measured: 2.7% faster on the 13M-cell river; on a mesh of a few rounds
// the hardware's own dispatch of one tile per block balances better)
inline int stage_grid(const swe_ctx *c, const void *kernel, int B, int ntiles)
{
    int gp = c->grid_persist;
    if (gp == 0) {
        const int res = resident_blocks(c, kernel, B);
        if (res > 0 && ntiles >= 8 * res) gp = res;
    }
    if (gp < 0) gp = 0;  // one tile per block, as asked
    return gp > 0 && gp < ntiles ? gp : ntiles;
}

// Fused pack of the high-overlap step: the send buffer the last stage fills
struct OverlapPlan {
    void *sendbuf = nullptr;  // null: a plain step
};

template <typename T>
int launch_step(swe_ctx *c, long long step, double dt_fixed, bool phi_force = false,
                const OverlapPlan &ov = OverlapPlan())
{
    using T4 = typename V4<T>::type;
    StageArgs<T> a{};
    a.n = c->n_total;
    a.n_scen = c->n_scen;
    a.nbr = (const int4 *)c->nbr;
    a.cell = (const T4 *)c->cell;
    a.man2 = (const T *)c->man2;
    a.he_geo = (const T4 *)c->he_geo;
    a.he_dist = (const T4 *)c->he_dist;
    a.he_co = (const T4 *)c->he_co;
    a.he_lam = (const T *)c->he_lam;
    a.he_gam = (const T *)c->he_gam;
    a.he_dfw = (const T *)c->he_dfw;
    a.he_nrm = (const typename V2<T>::type *)c->he_nrm;
    a.clock = c->clock;
    a.ncopy = c->ncopy;
    a.scen = c->scen;
    a.ser_t = c->ser_t;
    a.ser_q = c->ser_q;
    a.phi = c->phi;
    a.health = c->health;
    a.g = T(c->cfg.g);
    a.eps = T(c->cfg.eps);
    a.waf_pos = c->cfg.waf_positivity;
    a.cfl = c->cfg.cfl;
    a.dt_max = c->cfg.dt_max;
    a.dt_fixed = dt_fixed;
    a.cfl_rule = c->cfg.cfl_rule;
    a.slot_cur = (int)(step % 3);
    a.slot_next = (int)((step + 1) % 3);
    a.slot_reset = (int)((step + 2) % 3);
    // the one-thread-per-cell kernel is built for at most 256 threads, and
    // FP64 tiles stop at 256 cells (LDS)
    const bool euler = c->cfg.integrator == SWE_EULER;
    const bool cell_kernel = c->cfg.cell_kernel || (c->cfg.scheme == SWE_WAF && !euler);
    // the cell kernel, FP64 and the WAF tiles stop at 256 cells (FP64 WAF
    // tiles at 128: LDS)
    int B = cell_kernel || sizeof(T) == 8 || c->cfg.scheme == SWE_WAF ? std::min(c->block, 256) : c->block;
    if (c->cfg.scheme == SWE_WAF && !cell_kernel && sizeof(T) == 8) B = std::min(B, 128);
    KernelFn<T> k = pick_kernel<T>(c->cfg.scheme, c->cfg.limiter, c->cfg.waf_limiter, B,
                                   cell_kernel, seven_waves<T>(c, B), euler);
    const int ntiles = (c->n_total + B - 1) / B;
    dim3 grid(cell_kernel ? ntiles : stage_grid(c, (const void *)k, B, ntiles));
    const dim3 blk(B);
    T4 *Ucur = (T4 *)c->U[step & 1];
    // the learned limiter's phi is evaluated from U^n of the steps whose
    // index is a multiple of phi_every (every step by default; a step between
    // reuses the stored phi): by a kernel of its own ahead of the step, or
    // (when the configuration asks for it, tiled kernel only) by the step's
    // first stage.  phi_every divides the graph's period, so a captured
    // chunk, whose first step is aligned to it, evaluates on the same steps.
    const bool learned = c->cfg.scheme == SWE_MUSCL && c->cfg.limiter == SWE_LEARNED;
    const long long pe = c->cfg.phi_every > 1 ? c->cfg.phi_every : 1;
    const bool phi_now = learned && (phi_force || step % pe == 0);
    const bool phi_sep = phi_now && (cell_kernel || !c->cfg.phi_in_stage);
    a.mlp = (const MlpDev *)c->mlp;
    if (phi_sep && launch_limiter_phi(c, Ucur, c->phi) != SWE_OK) return SWE_ERR_DEVICE;
    KernelFn<T> k1 = k;  // the step's first stage
    dim3 grid1 = grid;
    if (phi_now && !phi_sep) {
        k1 = pick_kernel<T>(c->cfg.scheme, kLearnedNet, c->cfg.waf_limiter, B, 0, false, euler);
        grid1 = dim3(stage_grid(c, (const void *)k1, B, ntiles));
    }
    if (c->cfg.integrator == SWE_RK2) {
        // stage 1: U^n -> U1;  stage 2: U1 -> U^{n+1} = (U^n + E(U1)) / 2
        a.kind = 1; a.Uin = Ucur; a.U0 = Ucur; a.Uout = (T4 *)c->U1;
        hipLaunchKernelGGL(k1, grid1, blk, 0, c->stream, a);
        a.kind = 2; a.Uin = (T4 *)c->U1; a.U0 = Ucur; a.Uout = (T4 *)c->U[(step + 1) & 1];
    } else {
        a.kind = 0; a.Uin = Ucur; a.U0 = Ucur; a.Uout = (T4 *)c->U[(step + 1) & 1];
        k = k1;
        grid = grid1;
    }
    if (ov.sendbuf && c->n_send > 0) {  // the last stage also fills the send buffer
        a.pk_off = c->pk_off;
        a.pk_ent = c->pk_ent;
        a.pk_buf = (T *)ov.sendbuf;
        a.pk_ncell = c->send_prefix;
        a.pk_nsend = c->n_send;
    }
    hipLaunchKernelGGL(k, grid, blk, 0, c->stream, a);
    HIP_OK(c, hipGetLastError());
    return SWE_OK;
}

int launch_step_any(swe_ctx *c, long long step, double dt_fixed, bool phi_force = false)
{
    return c->cfg.precision == SWE_F64 ? launch_step<double>(c, step, dt_fixed, phi_force)
                                       : launch_step<float>(c, step, dt_fixed, phi_force);
}

int health_status(swe_ctx *c)
{
    int bits = 0;
    HIP_OK(c, hipMemcpy(&bits, c->health, sizeof(int), hipMemcpyDeviceToHost));
    if (bits & kHealthNonfinite) return set_err(c, SWE_ERR_NONFINITE, "non-finite value in the state");
    if (bits & kHealthNegDepth) return set_err(c, SWE_ERR_NEGATIVE_DEPTH, "depth below -eps in the state");
    return SWE_OK;
}

}  // namespace

extern "C" {

void swe_config_default(swe_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->abi_version = SWE_ABI_VERSION;
    cfg->precision = SWE_F32;
    cfg->scheme = SWE_MUSCL;
    cfg->integrator = SWE_RK2;
    cfg->limiter = SWE_MINMOD;
    cfg->waf_limiter = SWE_WAF_SUPERBEE;
    cfg->g = 9.81;
    cfg->cfl = 0.45;
    cfg->eps = 1e-6;
    cfg->dt_max = 0.0;
    cfg->waf_positivity = 1;
}

const char *swe_strerror(int code)
{
    switch (code) {
    case SWE_OK: return "ok";
    case SWE_ERR_ARG: return "invalid argument";
    case SWE_ERR_MESH: return "invalid mesh";
    case SWE_ERR_STATE: return "invalid or missing state";
    case SWE_ERR_NONFINITE: return "non-finite state";
    case SWE_ERR_NEGATIVE_DEPTH: return "negative depth";
    case SWE_ERR_DEVICE: return "HIP runtime error";
    case SWE_ERR_OOM: return "out of device memory";
    case SWE_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown error";
    }
}

const char *swe_last_error(const swe_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int swe_create(const swe_config *cfg, swe_ctx **out)
{
    if (!cfg || !out) return SWE_ERR_ARG;
    *out = nullptr;
    if (cfg->abi_version != SWE_ABI_VERSION) return SWE_ERR_ARG;
    if (cfg->precision != SWE_F32 && cfg->precision != SWE_F64) return SWE_ERR_ARG;
    if (cfg->scheme < 0 || cfg->scheme > 2 || cfg->integrator < 0 || cfg->integrator > 1 ||
        cfg->limiter < 0 || cfg->limiter > 4 || cfg->waf_limiter < 0 || cfg->waf_limiter > 2 ||
        cfg->cfl_rule < 0 || cfg->cfl_rule > 1 || !(cfg->g > 0) || !(cfg->cfl > 0) ||
        !(cfg->eps >= 0) || (cfg->waf_positivity != 0 && cfg->waf_positivity != 1) ||
        (cfg->phi_in_stage != 0 && cfg->phi_in_stage != 1) ||
        (cfg->phi_every != 0 && cfg->phi_every != 1 && cfg->phi_every != 2 && cfg->phi_every != 3 &&
         cfg->phi_every != 6) ||
        (cfg->block != 0 && cfg->block != 64 && cfg->block != 128 && cfg->block != 256 &&
         cfg->block != 512) ||
        cfg->cell_kernel < 0 || cfg->cell_kernel > 1 ||
        (cfg->waves != 0 && cfg->waves != 6 && cfg->waves != 7) || (!cfg->alloc != !cfg->free))
        return SWE_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SWE_ERR_DEVICE;
    if (cfg->device < 0 || cfg->device >= ndev) return SWE_ERR_ARG;
    auto *c = new swe_ctx;
    c->cfg = *cfg;
    c->dev = cfg->device;
    c->tsize = cfg->precision == SWE_F64 ? 8 : 4;
    // default tile: 256 cells, 64 for the FP32 tiled WAF kernel (its LDS
    // per cell is larger, and smaller tiles keep more of them in flight)
    const bool waf_tiled32 = cfg->scheme == SWE_WAF && cfg->integrator == SWE_EULER &&
                             !cfg->cell_kernel && cfg->precision == SWE_F32;
    c->block = cfg->block ? cfg->block : (waf_tiled32 ? 64 : 256);
    c->waves = cfg->waves;
    c->own_stream = cfg->stream == nullptr;
    if (!c->own_stream) c->stream = (hipStream_t)cfg->stream;
    if (hipSetDevice(c->dev) != hipSuccess ||
        (c->own_stream && hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        dalloc(c, (void **)&c->health, sizeof(int)) != hipSuccess ||
        dalloc(c, (void **)&c->flag, sizeof(int)) != hipSuccess ||
        hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->dev) != hipSuccess) {
        swe_destroy(c);
        return SWE_ERR_DEVICE;
    }
    (void)hipMemset(c->health, 0, sizeof(int));
    *out = c;
    return SWE_OK;
}

void swe_destroy(swe_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->dev);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release_mesh(c);
    dfree(c, c->mlp);
    dfree_t(c, c->health);
    dfree_t(c, c->flag);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->stream && c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"

namespace {

// Upload one mesh (a sub-domain with ghosts) or several independent meshes
// (a batch: one scenario each, concatenated, no ghosts).
int upload_meshes(swe_ctx *c, const swe_mesh *ms, int nm)
{
    if (!c || !ms || nm <= 0 || nm > kMaxScenarios) return set_err(c, SWE_ERR_ARG, "bad argument");
    HIP_OK(c, hipSetDevice(c->dev));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    // sizes first, before any array is read
    std::vector<int> off(nm + 1, 0);
    for (int i = 0; i < nm; ++i) {
        if (ms[i].n_total <= 0)
            return set_err(c, SWE_ERR_MESH, nm > 1 ? "mesh " + std::to_string(i) + ": no cells" : "mesh: no cells");
        if ((long long)off[i] + ms[i].n_total > 0x7fffffffLL / 3)
            return set_err(c, SWE_ERR_MESH, "too many cells");
        off[i + 1] = off[i] + ms[i].n_total;
    }
    // the stage kernels address every per-cell array with 32-bit byte
    // offsets; the largest is the half-edge set, 12 values per cell
    if ((unsigned long long)off[nm] * 12ull * c->tsize >= (1ull << 32))
        return set_err(c, SWE_ERR_UNSUPPORTED, "too many cells for one context (a per-cell array would exceed 4 GiB)");
    std::vector<HostGeometry> gs(nm);
    for (int i = 0; i < nm; ++i) {
        std::string msg;
        int rc = prepare_geometry(ms[i], i, gs[i], msg);
        if (rc != SWE_OK) return set_err(c, rc, nm > 1 ? "mesh " + std::to_string(i) + ": " + msg : msg);
    }
    const swe_mesh *m = &ms[0];
    const int n_ghost = nm == 1 ? m->n_total - m->n_owned : 0;
    int n_send = 0;
    if (nm > 1) {
        for (int i = 0; i < nm; ++i)
            if (ms[i].n_peers != 0 || ms[i].n_owned != ms[i].n_total)
                return set_err(c, SWE_ERR_MESH, "batched meshes cannot have ghost cells");
    } else {
        if (m->n_peers < 0) return set_err(c, SWE_ERR_MESH, "n_peers < 0");
        if (m->n_peers > 0) {
            if (!m->recv_off || !m->send_off || !m->send_idx)
                return set_err(c, SWE_ERR_MESH, "ghost lists missing");
            if (m->recv_off[0] != 0 || m->send_off[0] != 0 || m->recv_off[m->n_peers] != n_ghost)
                return set_err(c, SWE_ERR_MESH, "receive ranges do not cover the ghost cells");
            for (int j = 0; j < m->n_peers; ++j)
                if (m->recv_off[j + 1] < m->recv_off[j] || m->send_off[j + 1] < m->send_off[j])
                    return set_err(c, SWE_ERR_MESH, "ghost offsets not ascending");
            n_send = m->send_off[m->n_peers];
            for (int i = 0; i < n_send; ++i)
                if (m->send_idx[i] < 0 || m->send_idx[i] >= m->n_owned)
                    return set_err(c, SWE_ERR_MESH, "send index outside the owned cells");
        }
    }
    // concatenate (neighbour indices shifted by the mesh offset)
    HostGeometry g;
    if (nm == 1) {
        g = std::move(gs[0]);
    } else {
        const size_t N = off[nm];
        g.cell.reserve(4 * N); g.he_geo.reserve(12 * N); g.he_dist.reserve(12 * N); g.nbr4.reserve(4 * N);
        for (int i = 0; i < nm; ++i) {
            HostGeometry &gi = gs[i];
            g.cell.insert(g.cell.end(), gi.cell.begin(), gi.cell.end());
            g.he_geo.insert(g.he_geo.end(), gi.he_geo.begin(), gi.he_geo.end());
            g.he_dist.insert(g.he_dist.end(), gi.he_dist.begin(), gi.he_dist.end());
            for (size_t j = 0; j < gi.nbr4.size(); ++j) {
                int32_t v = gi.nbr4[j];
                if ((j & 3) != 3 && v >= 0) v += off[i];
                g.nbr4.push_back(v);
            }
            std::vector<double>().swap(gi.cell);
            std::vector<double>().swap(gi.he_geo);
            std::vector<double>().swap(gi.he_dist);
        }
    }
    release_mesh(c);
    c->n_total = off[nm];
    c->n_owned = nm == 1 ? m->n_owned : c->n_total;
    c->n_scen = nm;
    c->n_send = n_send;
    c->send_prefix = 0;
    for (int i = 0; i < n_send; ++i) c->send_prefix = std::max(c->send_prefix, m->send_idx[i] + 1);
    c->n_ghost = n_ghost;
    c->scen_off = off;
    int rc = c->cfg.precision == SWE_F64 ? upload_geometry<double>(c, g) : upload_geometry<float>(c, g);
    if (rc != SWE_OK) return rc;
    const size_t n = c->n_total, ts = c->tsize;
    HIP_OK(c, dalloc(c, (void **)&c->U[0], 4 * ts * n));
    HIP_OK(c, dalloc(c, (void **)&c->U[1], 4 * ts * n));
    HIP_OK(c, dalloc(c, (void **)&c->U1, 4 * ts * n));
    HIP_OK(c, dalloc(c, (void **)&c->tmp3, 3 * ts * n));
    HIP_OK(c, dalloc(c, (void **)&c->bed, ts * n));
    HIP_OK(c, dalloc(c, (void **)&c->phi, sizeof(float) * 3 * n));
    // CFL partial copies: enough lines that concurrent block commits rarely
    // meet on one, few enough that large batches stay small
    c->ncopy = nm <= 64 ? 16 : (nm <= 1024 ? 8 : 4);
    HIP_OK(c, dalloc(c, (void **)&c->clock, clock_bytes(c)));
    HIP_OK(c, dalloc(c, (void **)&c->t0, sizeof(double) * (size_t)nm));
    {
        std::vector<double> bd(n);
        for (int i = 0; i < nm; ++i) std::copy(ms[i].cell_b, ms[i].cell_b + ms[i].n_total, bd.begin() + off[i]);
        if (ts == 8) {
            HIP_OK(c, hipMemcpy(c->bed, bd.data(), 8 * n, hipMemcpyHostToDevice));
        } else {
            std::vector<float> bf(bd.begin(), bd.end());
            HIP_OK(c, hipMemcpy(c->bed, bf.data(), 4 * n, hipMemcpyHostToDevice));
        }
    }
    if (n_send > 0) {
        HIP_OK(c, dalloc(c, (void **)&c->send_idx, sizeof(int) * n_send));
        HIP_OK(c, hipMemcpy(c->send_idx, m->send_idx, sizeof(int) * n_send, hipMemcpyHostToDevice));
        // send entries of each send cell (CSR over cells [0, send_prefix)),
        // for the pack fused into the last stage of a high-overlap step
        std::vector<int> off(c->send_prefix + 1, 0), ent(n_send);
        for (int i = 0; i < n_send; ++i) off[m->send_idx[i] + 1]++;
        for (int i = 0; i < c->send_prefix; ++i) off[i + 1] += off[i];
        std::vector<int> fill(off.begin(), off.end() - 1);
        for (int i = 0; i < n_send; ++i) ent[fill[m->send_idx[i]]++] = i;
        HIP_OK(c, dalloc(c, (void **)&c->pk_off, sizeof(int) * (c->send_prefix + 1)));
        HIP_OK(c, dalloc(c, (void **)&c->pk_ent, sizeof(int) * n_send));
        HIP_OK(c, hipMemcpy(c->pk_off, off.data(), sizeof(int) * (c->send_prefix + 1), hipMemcpyHostToDevice));
        HIP_OK(c, hipMemcpy(c->pk_ent, ent.data(), sizeof(int) * n_send, hipMemcpyHostToDevice));
    }
    c->h_scen.assign(nm, ScenParams{});
    c->series.assign(nm, {});
    for (int i = 0; i < nm; ++i) {
        const double L = ms[i].inflow_length > 0 ? ms[i].inflow_length
                                                 : (nm == 1 ? g.inflow_length : gs[i].inflow_length);
        ScenParams &sp = c->h_scen[i];
        sp.inflow_q = ms[i].inflow_q;
        sp.inv_inflow_len = L > 0 ? 1.0 / L : 0.0;
        sp.outflow_stage = ms[i].outflow_stage;
    }
    rc = push_scenarios(c);
    if (rc != SWE_OK) return rc;
    c->has_mesh = true;
    c->has_state = false;
    c->tuned = false;
    return SWE_OK;
}

}  // namespace

extern "C" {

int swe_mesh_upload(swe_ctx *c, const swe_mesh *m) { return upload_meshes(c, m, 1); }

int swe_mesh_upload_batch(swe_ctx *c, int n_meshes, const swe_mesh *meshes)
{
    return upload_meshes(c, meshes, n_meshes);
}

int swe_set_bc_series_scenario(swe_ctx *c, int scen, int n, const double *t, const double *q)
{
    if (!c || n < 0 || (n > 0 && (!t || !q))) return set_err(c, SWE_ERR_ARG, "bad series");
    if (!c->has_mesh) return set_err(c, SWE_ERR_STATE, "no mesh");
    if (scen < 0 || scen >= c->n_scen) return set_err(c, SWE_ERR_ARG, "scenario index");
    for (int i = 0; i + 1 < n; ++i)
        if (!(t[i + 1] > t[i])) return set_err(c, SWE_ERR_ARG, "series times must increase");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->series[scen].first.assign(t, t + n);
    c->series[scen].second.assign(q, q + n);
    if (c->graph) { (void)hipGraphExecDestroy(c->graph); c->graph = nullptr; }
    return push_scenarios(c);
}

int swe_set_bc_series(swe_ctx *c, int n, const double *t, const double *q)
{
    return swe_set_bc_series_scenario(c, 0, n, t, q);
}

int swe_batch_offsets(const swe_ctx *c, int32_t *n_scen, int32_t *offsets)
{
    if (!c || !n_scen) return SWE_ERR_ARG;
    *n_scen = c->n_scen;
    if (offsets)
        for (int i = 0; i <= c->n_scen; ++i) offsets[i] = c->scen_off.empty() ? 0 : c->scen_off[i];
    return SWE_OK;
}

int swe_scenario_times(swe_ctx *c, double *t)
{
    if (!c || !t) return set_err(c, SWE_ERR_ARG, "null");
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    std::vector<ClockWord> k(clock_bytes(c) / sizeof(ClockWord));
    HIP_OK(c, hipMemcpy(k.data(), c->clock, clock_bytes(c), hipMemcpyDeviceToHost));
    for (int s = 0; s < c->n_scen; ++s)
        std::memcpy(&t[s], &k[clock_off(c->ncopy, s, (int)(c->step_count % 3))], sizeof(double));
    return health_status(c);
}

int swe_set_state(swe_ctx *c, const void *h, const void *hu, const void *hv, int where, double t)
{
    if (!c || !h || !hu || !hv || (where != SWE_HOST && where != SWE_DEVICE))
        return set_err(c, SWE_ERR_ARG, "bad argument");
    if (!c->has_mesh) return set_err(c, SWE_ERR_STATE, "no mesh uploaded");
    HIP_OK(c, hipSetDevice(c->dev));
    const size_t n = c->n_total, ts = c->tsize;
    char *tmp = (char *)c->tmp3;
    const hipMemcpyKind kind = where == SWE_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIP_OK(c, hipMemcpyAsync(tmp, h, ts * n, kind, c->stream));
    HIP_OK(c, hipMemcpyAsync(tmp + ts * n, hu, ts * n, kind, c->stream));
    HIP_OK(c, hipMemcpyAsync(tmp + 2 * ts * n, hv, ts * n, kind, c->stream));
    HIP_OK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    HIP_OK(c, hipMemsetAsync(c->health, 0, sizeof(int), c->stream));
    const int B = 256, G = (int)((n + B - 1) / B);
    if (ts == 8)
        hipLaunchKernelGGL(k_pack_state<double>, dim3(G), dim3(B), 0, c->stream, (int)n,
                           (const double *)tmp, (const double *)(tmp + 8 * n),
                           (const double *)(tmp + 16 * n), (const double *)c->bed,
                           (double4 *)c->U[0], c->flag, c->cfg.eps);
    else
        hipLaunchKernelGGL(k_pack_state<float>, dim3(G), dim3(B), 0, c->stream, (int)n,
                           (const float *)tmp, (const float *)(tmp + 4 * n),
                           (const float *)(tmp + 8 * n), (const float *)c->bed, (float4 *)c->U[0],
                           c->flag, (float)c->cfg.eps);
    HIP_OK(c, hipGetLastError());
    int bad = 0;
    HIP_OK(c, hipMemcpyAsync(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (bad) return set_err(c, SWE_ERR_STATE, "state has a negative or non-finite value");
    c->step_count = 0;
    int rc = init_clock(c, t);
    if (rc != SWE_OK) return rc;
    c->has_state = true;
    return SWE_OK;
}

}  // extern "C"

namespace swe {

int init_clock(swe_ctx *c, double t)
{
    const size_t n = c->n_total, ts = c->tsize;
    const int B = 256, G = (int)((n + B - 1) / B);
    c->h_t0.assign(c->n_scen, t);
    HIP_OK(c, hipMemcpyAsync(c->t0, c->h_t0.data(), sizeof(double) * c->n_scen,
                             hipMemcpyHostToDevice, c->stream));
    // slot 0: time and CFL minima of the initial state; slot 1 cleared
    const int gs = (c->n_scen * c->ncopy + 255) / 256;
    hipLaunchKernelGGL(k_clock_reset, dim3(gs), dim3(256), 0, c->stream, c->clock, c->ncopy, c->n_scen,
                       0, c->t0, 1);
    hipLaunchKernelGGL(k_clock_reset, dim3(gs), dim3(256), 0, c->stream, c->clock, c->ncopy, c->n_scen,
                       1, c->t0, 0);
    if (ts == 8)
        hipLaunchKernelGGL(k_cfl_init<double>, dim3(G), dim3(B), 0, c->stream, (int)n,
                           (const int4 *)c->nbr, (const double4 *)c->cell,
                           (const double4 *)c->U[0], c->clock, c->ncopy, 0, c->cfg.cfl_rule,
                           c->cfg.g, c->cfg.eps);
    else
        hipLaunchKernelGGL(k_cfl_init<float>, dim3(G), dim3(B), 0, c->stream, (int)n,
                           (const int4 *)c->nbr, (const float4 *)c->cell, (const float4 *)c->U[0],
                           c->clock, c->ncopy, 0, c->cfg.cfl_rule, (float)c->cfg.g,
                           (float)c->cfg.eps);
    HIP_OK(c, hipGetLastError());
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->has_state = true;
    return SWE_OK;
}

}  // namespace swe

extern "C" {

int swe_read_state(swe_ctx *c, void *h, void *hu, void *hv, int where)
{
    if (!c || !h || !hu || !hv || (where != SWE_HOST && where != SWE_DEVICE))
        return set_err(c, SWE_ERR_ARG, "bad argument");
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    HIP_OK(c, hipSetDevice(c->dev));
    const size_t n = c->n_total, ts = c->tsize;
    char *tmp = (char *)c->tmp3;
    const int B = 256, G = (int)((n + B - 1) / B);
    void *Ucur = c->U[c->step_count & 1];
    if (ts == 8)
        hipLaunchKernelGGL(k_unpack_state<double>, dim3(G), dim3(B), 0, c->stream, (int)n,
                           (const double4 *)Ucur, (double *)tmp, (double *)(tmp + 8 * n),
                           (double *)(tmp + 16 * n));
    else
        hipLaunchKernelGGL(k_unpack_state<float>, dim3(G), dim3(B), 0, c->stream, (int)n,
                           (const float4 *)Ucur, (float *)tmp, (float *)(tmp + 4 * n),
                           (float *)(tmp + 8 * n));
    HIP_OK(c, hipGetLastError());
    const hipMemcpyKind kind = where == SWE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIP_OK(c, hipMemcpyAsync(h, tmp, ts * n, kind, c->stream));
    HIP_OK(c, hipMemcpyAsync(hu, tmp + ts * n, ts * n, kind, c->stream));
    HIP_OK(c, hipMemcpyAsync(hv, tmp + 2 * ts * n, ts * n, kind, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return health_status(c);
}

// true if p is device (or managed) memory of the context's device; a failed
// query leaves HIP's last error set, which is cleared here so that the next
// launch check does not report it
static bool device_buffer(const swe_ctx *c, const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == c->dev;
}

int swe_snapshot(swe_ctx *c, void *h, void *hu, void *hv, void *done_event)
{
    if (!c || !h || !hu || !hv) return set_err(c, SWE_ERR_ARG, "bad argument");
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    HIP_OK(c, hipSetDevice(c->dev));
    if (!device_buffer(c, h) || !device_buffer(c, hu) || !device_buffer(c, hv))
        return set_err(c, SWE_ERR_ARG, "snapshot buffers must be device memory of the context's device");
    const size_t n = c->n_total;
    const int B = 256, G = (int)((n + B - 1) / B);
    void *Ucur = c->U[c->step_count & 1];
    if (c->tsize == 8)
        hipLaunchKernelGGL(k_unpack_state<double>, dim3(G), dim3(B), 0, c->stream, (int)n,
                           (const double4 *)Ucur, (double *)h, (double *)hu, (double *)hv);
    else
        hipLaunchKernelGGL(k_unpack_state<float>, dim3(G), dim3(B), 0, c->stream, (int)n,
                           (const float4 *)Ucur, (float *)h, (float *)hu, (float *)hv);
    HIP_OK(c, hipGetLastError());
    if (done_event) HIP_OK(c, hipEventRecord((hipEvent_t)done_event, c->stream));
    return SWE_OK;
}

// Capture and instantiate the graph of kGraphSteps steps (the period of the
// clock slots and of the state buffers, so one graph serves every aligned
// run of steps) for this dt_fixed, unless it exists.  Nothing is launched.
static int ensure_graph(swe_ctx *c, double dt_fixed)
{
    if (c->graph && c->graph_dt == dt_fixed) return SWE_OK;
    if (c->graph) { (void)hipGraphExecDestroy(c->graph); c->graph = nullptr; }
    hipGraph_t gr = nullptr;
    HIP_OK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = SWE_OK;
    for (int s = 0; s < kGraphSteps && rc == SWE_OK; ++s) rc = launch_step_any(c, s, dt_fixed);
    hipError_t e = hipStreamEndCapture(c->stream, &gr);
    if (rc != SWE_OK) { if (gr) (void)hipGraphDestroy(gr); return rc; }
    if (e != hipSuccess) return set_err(c, SWE_ERR_DEVICE, "graph capture failed");
    e = hipGraphInstantiate(&c->graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) { c->graph = nullptr; return set_err(c, SWE_ERR_DEVICE, "graph instantiation failed"); }
    c->graph_dt = dt_fixed;
    return SWE_OK;
}

static int step_ready(swe_ctx *c)
{
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    if (c->cfg.scheme == SWE_MUSCL && c->cfg.limiter == SWE_LEARNED && !c->has_mlp)
        return set_err(c, SWE_ERR_STATE, "learned limiter weights not set");
    return SWE_OK;
}

int swe_step_kernel(const swe_ctx *c, const char **name, int *launches_per_step)
{
    if (!c || !name || !launches_per_step) return SWE_ERR_ARG;
    const bool euler = c->cfg.integrator == SWE_EULER;
    const bool cell_kernel = c->cfg.cell_kernel || (c->cfg.scheme == SWE_WAF && !euler);
    const bool learned = c->cfg.scheme == SWE_MUSCL && c->cfg.limiter == SWE_LEARNED;
    const int stages = euler ? 1 : 2;
    if (cell_kernel) *name = "k_stage";
    else if (c->cfg.scheme == SWE_WAF) *name = "k_stage_tiled_waf";
    else *name = learned && !c->cfg.phi_in_stage ? "k_stage_tiled+k_limiter_phi" : "k_stage_tiled";
    *launches_per_step = stages + (learned && (cell_kernel || !c->cfg.phi_in_stage) ? 1 : 0);
    return SWE_OK;
}

int swe_prepare(swe_ctx *c, double dt_fixed)
{
    if (!c) return SWE_ERR_ARG;
    const int rc = step_ready(c);
    if (rc != SWE_OK) return rc;
    HIP_OK(c, hipSetDevice(c->dev));
    if (!(dt_fixed > 0.0)) dt_fixed = 0.0;
    return c->use_graphs ? ensure_graph(c, dt_fixed) : SWE_OK;
}

int swe_step(swe_ctx *c, int n_steps, double dt_fixed)
{
    if (!c || n_steps < 0) return set_err(c, SWE_ERR_ARG, "bad argument");
    const int ready = step_ready(c);
    if (ready != SWE_OK) return ready;
    HIP_OK(c, hipSetDevice(c->dev));
    if (!(dt_fixed > 0.0)) dt_fixed = 0.0;
    HIP_OK(c, hipEventRecord(c->ev0, c->stream));
    int done = 0;
    while (done < n_steps) {
        const bool aligned = (c->step_count % kGraphSteps) == 0;
        if (c->use_graphs && aligned && n_steps - done >= kGraphSteps) {
            const int rc = ensure_graph(c, dt_fixed);
            if (rc != SWE_OK) return rc;
            HIP_OK(c, hipGraphLaunch(c->graph, c->stream));
            c->phi_stale = false;  // the chunk's first step evaluates phi
            c->step_count += kGraphSteps;
            done += kGraphSteps;
        } else {
            int rc = launch_step_any(c, c->step_count, dt_fixed, c->phi_stale);
            if (rc != SWE_OK) return rc;
            c->phi_stale = false;
            c->step_count += 1;
            done += 1;
        }
    }
    HIP_OK(c, hipEventRecord(c->ev1, c->stream));
    c->ran = true;
    return SWE_OK;
}

int swe_step_overlap(swe_ctx *c, double dt_fixed, void *dev_sendbuf, void *pack_done_event)
{
    if (!c) return SWE_ERR_ARG;
    if (!dev_sendbuf && c->n_send > 0) return set_err(c, SWE_ERR_ARG, "null send buffer");
    const int ready = step_ready(c);
    if (ready != SWE_OK) return ready;
    HIP_OK(c, hipSetDevice(c->dev));
    if (!(dt_fixed > 0.0)) dt_fixed = 0.0;
    HIP_OK(c, hipEventRecord(c->ev0, c->stream));
    OverlapPlan ov;
    ov.sendbuf = dev_sendbuf;
    const int rc = c->cfg.precision == SWE_F64 ? launch_step<double>(c, c->step_count, dt_fixed, c->phi_stale, ov)
                                               : launch_step<float>(c, c->step_count, dt_fixed, c->phi_stale, ov);
    if (rc != SWE_OK) return rc;
    c->phi_stale = false;
    if (pack_done_event) HIP_OK(c, hipEventRecord((hipEvent_t)pack_done_event, c->stream));
    c->step_count += 1;
    HIP_OK(c, hipEventRecord(c->ev1, c->stream));
    c->ran = true;
    return SWE_OK;
}

int swe_autotune(swe_ctx *c, int n_steps, int *block_out, int *grid_out)
{
    if (!c || n_steps <= 0) return set_err(c, SWE_ERR_ARG, "bad argument");
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    HIP_OK(c, hipSetDevice(c->dev));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    int ncu = 0;
    HIP_OK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->dev));
    // save the state, clocks and step index; every candidate starts from them
    const size_t bytes = 4 * c->tsize * (size_t)c->n_total;
    void *saveU = nullptr;
    void *saveK = nullptr;
    HIP_OK(c, dalloc(c, &saveU, bytes));
    if (dalloc(c, &saveK, clock_bytes(c)) != hipSuccess) {
        dfree(c, saveU);
        return set_err(c, SWE_ERR_OOM, "autotune buffers");
    }
    const long long step0 = c->step_count;
    void *Ucur = c->U[step0 & 1];
    HIP_OK(c, hipMemcpyAsync(saveU, Ucur, bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(saveK, c->clock, clock_bytes(c), hipMemcpyDeviceToDevice, c->stream));
    const bool graphs = c->use_graphs;
    c->use_graphs = false;
    float best = 1e30f;
    int best_b = c->block, best_g = c->grid_persist, best_w = c->waves;
    int rc = SWE_OK;
    // only launch shapes of the configured kernel: they give bitwise the same
    // results (the tiled kernel is tiling-independent), the two kernels do not
    const int cell0 = c->cfg.cell_kernel;
    const bool tiled = c->cfg.scheme != SWE_WAF && !cell0;
    const bool f64 = c->cfg.precision == SWE_F64;
    int best_cell = cell0;
    const bool learned = c->cfg.scheme == SWE_MUSCL && c->cfg.limiter == SWE_LEARNED;
    for (int B : {64, 128, 256, 512})
    for (int W : {6, 7}) {
        if (B == 512 && (!tiled || f64)) continue;  // FP32 tiled kernel only
        // a second register budget only for the FP32 tiled kernel with 256-cell tiles
        if (W == 7 && (B != 256 || !tiled || f64 || learned)) continue;
        for (int persist = 0; persist < 2 && rc == SWE_OK; ++persist) {
            c->block = B;
            c->waves = W;
            c->grid_persist = -1;  // one tile per block
            if (persist) {
                const bool cell = c->cfg.cell_kernel || (c->cfg.scheme == SWE_WAF && c->cfg.integrator != SWE_EULER);
                const int res = c->cfg.precision == SWE_F64
                                    ? resident_blocks(c, (const void *)pick_kernel<double>(c->cfg.scheme, c->cfg.limiter, c->cfg.waf_limiter, B, cell, false, c->cfg.integrator == SWE_EULER), B)
                                    : resident_blocks(c, (const void *)pick_kernel<float>(c->cfg.scheme, c->cfg.limiter, c->cfg.waf_limiter, B, cell, W == 7, c->cfg.integrator == SWE_EULER), B);
                c->grid_persist = res > 0 ? res : ncu * (2048 / B);
            }
            (void)hipMemcpyAsync(Ucur, saveU, bytes, hipMemcpyDeviceToDevice, c->stream);
            (void)hipMemcpyAsync(c->clock, saveK, clock_bytes(c), hipMemcpyDeviceToDevice, c->stream);
            c->step_count = step0;
            c->phi_stale = true;
            rc = swe_step(c, 2, 0.0);  // warm-up
            if (rc != SWE_OK) break;
            rc = swe_step(c, n_steps, 0.0);
            if (rc != SWE_OK) break;
            float ms = 0.f;
            rc = swe_last_step_ms(c, &ms);
            if (rc == SWE_OK && ms < best) {
                best = ms; best_b = B; best_g = c->grid_persist; best_cell = c->cfg.cell_kernel;
                best_w = W;
            }
        }
    }
    c->use_graphs = graphs;
    c->block = best_b;
    c->grid_persist = best_g;
    c->waves = best_w;
    c->cfg.cell_kernel = best_cell;
    (void)hipMemcpyAsync(Ucur, saveU, bytes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->clock, saveK, clock_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    c->step_count = step0;
    c->phi_stale = true;  // phi was overwritten by the candidates' runs
    dfree(c, saveU);
    dfree(c, saveK);
    if (c->graph) { (void)hipGraphExecDestroy(c->graph); c->graph = nullptr; }
    if (rc != SWE_OK) return rc;
    c->tuned = true;
    if (block_out) *block_out = best_b;
    if (grid_out) *grid_out = best_g;
    return SWE_OK;
}

int swe_sync(swe_ctx *c)
{
    if (!c) return SWE_ERR_ARG;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return c->has_state ? health_status(c) : SWE_OK;
}

int swe_health(swe_ctx *c, int *bits)
{
    if (!c || !bits) return set_err(c, SWE_ERR_ARG, "null");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    HIP_OK(c, hipMemcpy(bits, c->health, sizeof(int), hipMemcpyDeviceToHost));
    return SWE_OK;
}

int swe_time(swe_ctx *c, double *t)
{
    if (!c || !t) return set_err(c, SWE_ERR_ARG, "null");
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    HIP_OK(c, hipMemcpy(t, c->clock + clock_off(c->ncopy, 0, (int)(c->step_count % 3)),
                        sizeof(double), hipMemcpyDeviceToHost));
    return health_status(c);
}

int swe_local_dt(swe_ctx *c, double *dt)
{
    if (!c || !dt) return set_err(c, SWE_ERR_ARG, "null");
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    // reduce the copies of scenario 0's current slot, as the kernels do
    const int nc = c->ncopy;
    std::vector<ClockWord> k((size_t)(nc + 1) * kClockLine);
    HIP_OK(c, hipMemcpy(k.data(), c->clock + clock_off(nc, 0, (int)(c->step_count % 3)),
                        sizeof(ClockWord) * k.size(), hipMemcpyDeviceToHost));
    ClockWord mnb = kInfBits, mxb = 0ull;
    for (int j = 0; j < nc; ++j) {
        const ClockWord *q = &k[(size_t)(1 + j) * kClockLine];
        mnb = std::min(mnb, q[kCfqMin]);
        mxb = std::max(mxb, q[kCfqMax]);
    }
    double v;
    if (mnb == kInfBits) {  // nothing wet
        v = c->cfg.dt_max > 0 ? c->cfg.dt_max : 0.0;
    } else {
        double mn, mx;
        std::memcpy(&mn, &mnb, 8);
        std::memcpy(&mx, &mxb, 8);
        v = c->cfg.cfl_rule == 1 ? c->cfg.cfl * mn / mx : c->cfg.cfl * mn;
        if (c->cfg.dt_max > 0 && v > c->cfg.dt_max) v = c->cfg.dt_max;
    }
    *dt = v;
    return SWE_OK;
}

int swe_ghost_sizes(const swe_ctx *c, int32_t *n_send, int32_t *n_ghost)
{
    if (!c || !n_send || !n_ghost) return SWE_ERR_ARG;
    *n_send = c->n_send;
    *n_ghost = c->n_ghost;
    return SWE_OK;
}

int swe_pack_ghosts(swe_ctx *c, void *buf)
{
    if (!c || (!buf && c->n_send > 0)) return set_err(c, SWE_ERR_ARG, "null buffer");
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    if (c->n_send == 0) return SWE_OK;
    HIP_OK(c, hipSetDevice(c->dev));
    const int B = 256, G = (c->n_send + B - 1) / B;
    void *Ucur = c->U[c->step_count & 1];
    if (c->tsize == 8)
        hipLaunchKernelGGL(k_pack_ghosts<double>, dim3(G), dim3(B), 0, c->stream, c->n_send,
                           c->send_idx, (const double4 *)Ucur, (double *)buf);
    else
        hipLaunchKernelGGL(k_pack_ghosts<float>, dim3(G), dim3(B), 0, c->stream, c->n_send,
                           c->send_idx, (const float4 *)Ucur, (float *)buf);
    HIP_OK(c, hipGetLastError());
    return SWE_OK;
}

int swe_unpack_ghosts(swe_ctx *c, const void *buf)
{
    if (!c || (!buf && c->n_ghost > 0)) return set_err(c, SWE_ERR_ARG, "null buffer");
    if (!c->has_state) return set_err(c, SWE_ERR_STATE, "no state");
    if (c->n_ghost == 0) return SWE_OK;
    HIP_OK(c, hipSetDevice(c->dev));
    const int B = 256, G = (c->n_ghost + B - 1) / B;
    void *Ucur = c->U[c->step_count & 1];
    if (c->tsize == 8)
        hipLaunchKernelGGL(k_unpack_ghosts<double>, dim3(G), dim3(B), 0, c->stream, c->n_owned,
                           c->n_ghost, (const double *)buf, (double4 *)Ucur);
    else
        hipLaunchKernelGGL(k_unpack_ghosts<float>, dim3(G), dim3(B), 0, c->stream, c->n_owned,
                           c->n_ghost, (const float *)buf, (float4 *)Ucur);
    HIP_OK(c, hipGetLastError());
    return SWE_OK;
}

int swe_last_step_ms(swe_ctx *c, float *ms)
{
    if (!c || !ms) return SWE_ERR_ARG;
    if (!c->ran) return set_err(c, SWE_ERR_STATE, "no step yet");
    HIP_OK(c, hipEventSynchronize(c->ev1));
    HIP_OK(c, hipEventElapsedTime(ms, c->ev0, c->ev1));
    return SWE_OK;
}

}  // extern "C"
