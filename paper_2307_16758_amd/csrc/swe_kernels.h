// Device-side numerics of the shallow-water step (Delmas & Soulaimani,
// Sec. 6.1 - 6.2): interface reconstruction, hydrostatic reconstruction,
// HLLC / WAF fluxes and boundary fluxes, written once for float and double.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace swe {

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };
template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };

enum { kHLLC1 = 0, kMUSCL = 1, kWAF = 2 };
enum { kMinmod = 0, kSuperbee = 1, kVanAlbada = 2, kLearned = 3, kZeroSlope = 4 };
enum { kWafSuperbee = 0, kWafGodunov = 1, kWafUnlimited = 2 };
enum { kBcWall = -1, kBcTransmissive = -2, kBcInflow = -3, kBcOutflow = -4, kBcHalo = -5 };
enum { kHealthNonfinite = 1, kHealthNegDepth = 2, kHealthClipped = 4 };

// Per-scenario step clock, three slots per scenario rotating with the step
// index: the current step reads slot s, reduces the next CFL step into slot
// s+1 and clears slot s+2.  A slot is 1 + ncopy cache lines of 128 bytes:
// the time (double) in the first, then ncopy partials of the CFL quantities
// over wet owned cells: the minimum of R_i / lambda_i (rule 0) or of R_i
// (rule 1), and the maximum of lambda_i, as the bit patterns of non-negative
// doubles, whose integer order is their numeric order.  Blocks commit to
// copy (block index mod ncopy), so concurrent atomics spread over ncopy
// lines; readers reduce the copies.
constexpr int kClockLine = 16;  // 64-bit words per 128-byte line
enum { kCfqMin = 0, kCfqMax = 1 };

struct ScenParams {
    double inflow_q;         // constant total discharge
    double inv_inflow_len;   // 1 / total inflow edge length
    double outflow_stage;
    int series_off, series_n;  // hydrograph points in the series arrays
};

// Interface values of one half-edge: depth, bed, normal and tangential
// velocity, and the free surface eta = h + b as reconstructed.
template <typename T> struct Half { T h, b, un, ut, eta; };

// Division in the working precision: FP32 through the hardware reciprocal
// (1 ulp; denormals are flushed in this build), FP64 exact.
template <typename T> __device__ __forceinline__ T frcp(T x) { return T(1) / x; }
template <> __device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename T> __device__ __forceinline__ T fdiv(T a, T b) { return a / b; }
template <> __device__ __forceinline__ float fdiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// h^(-4/3) of the Manning term: FP32 as 2^(-4/3 log2 h) on the hardware
// log2 / exp2 (about 1e-6 relative), FP64 through cbrt.
template <typename T> __device__ __forceinline__ T pow_m43(T h) { return T(1) / (h * cbrt(h)); }
template <> __device__ __forceinline__ float pow_m43<float>(float h)
{
    return __builtin_amdgcn_exp2f(-1.3333333f * __builtin_amdgcn_logf(h));
}

template <typename T> __device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }
template <typename T> __device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }

// velocity of a cell state in the frame (n, t = rot90(n))
template <typename T, typename T4>
__device__ __forceinline__ void frame_vel(const T4 &U, T nx, T ny, T eps, T &un, T &ut)
{
    const T u = U.x > eps ? fdiv(U.y, U.x) : T(0);
    const T v = U.x > eps ? fdiv(U.z, U.x) : T(0);
    un = u * nx + v * ny;
    ut = -u * ny + v * nx;
}

// Slope limiters of Sec. 6.2.3: beta form branching on the sign of the jump
// across the edge (beta = 1 MINBEE, beta = 2 SUPERBEE), and van Albada.
template <typename T, int LIM>
__device__ __forceinline__ T limit(T sb, T sf)
{
    if (LIM == kVanAlbada) return sb * sf > T(0) ? fdiv(sb * sf * (sb + sf), sb * sb + sf * sf) : T(0);
    if (LIM == kZeroSlope) return T(0);
    const T beta = LIM == kSuperbee ? T(2) : T(1);
    if (sf > T(0)) return tmax(T(0), tmax(tmin(beta * sb, sf), tmin(sb, beta * sf)));
    if (sf < T(0)) return tmin(T(0), tmin(tmax(beta * sb, sf), tmax(sb, beta * sf)));
    return T(0);
}

// The learned limiter's slope s (phi times the central slope) kept inside
// the second-order TVD region of the backward and forward slopes sb, sf:
// zero unless they share a sign, else the sign of sf and at most
// 2 min(|sb|, |sf|) (Sweby's bound; phi = 1 gives the monotonized central
// limiter).  All three may carry the same positive factor (d_mid).
template <typename T> __device__ __forceinline__ T tvd_clip(T s, T sb, T sf)
{
    if constexpr (sizeof(T) == 4) {
        // by median selections: 2 minmod(sb, sf) is the bound, and s (the
        // scaled central slope, of the sign of sb and sf when they agree)
        // is clipped between it and zero
        return __builtin_amdgcn_fmed3f(s, 2.0f * __builtin_amdgcn_fmed3f(sb, sf, 0.0f), 0.0f);
    }
    const T lim = T(2) * tmin(fabs(sb), fabs(sf));
    return sb * sf > T(0) ? copysign(tmin(fabs(s), lim), sf) : T(0);
}

// Interface values of cell c across one of its edges, in c's outward-normal
// frame (Sec. 6.2.3 on the rotated states T_n U): h, b- and the normal and
// tangential velocities.  Uk is the cell across the edge, Ua / Ub the two
// other neighbours of c (upwind cells).  dist = (1/d_up, 1/d_fwd,
// 1/d_central, d_fwd).  First order unless the scheme is MUSCL, all stencil
// cells are wet, at least one upwind cell exists and h- >= 0.
template <typename T, typename T4, int SCHEME, int LIM>
__device__ __forceinline__ Half<T> reconstruct(const T4 &Uc, const T4 &Uk, const T4 &Ua, bool ha,
                                               const T4 &Ub, bool hb, T nx, T ny, T dm,
                                               const T4 &dist, float phi, T eps)
{
    Half<T> r;
    r.h = Uc.x;
    r.b = Uc.w;
    r.eta = Uc.x + Uc.w;
    frame_vel(Uc, nx, ny, eps, r.un, r.ut);
    if (SCHEME != kMUSCL) return r;
    if (!(Uc.x > eps) || !(Uk.x > eps)) return r;
    if ((ha && !(Ua.x > eps)) || (hb && !(Ub.x > eps)) || (!ha && !hb)) return r;
    T qc[4] = {Uc.x, Uc.x + Uc.w, r.un, r.ut};
    T qk[4];
    qk[0] = Uk.x;
    qk[1] = Uk.x + Uk.w;
    frame_vel(Uk, nx, ny, eps, qk[2], qk[3]);
    T qu[4];
    if (ha && hb) {
        T qa[4], qb[4];
        qa[0] = Ua.x; qa[1] = Ua.x + Ua.w; frame_vel(Ua, nx, ny, eps, qa[2], qa[3]);
        qb[0] = Ub.x; qb[1] = Ub.x + Ub.w; frame_vel(Ub, nx, ny, eps, qb[2], qb[3]);
#pragma unroll
        for (int i = 0; i < 4; ++i) qu[i] = T(0.5) * (qa[i] + qb[i]);
    } else {
        const T4 &Uo = ha ? Ua : Ub;
        qu[0] = Uo.x; qu[1] = Uo.x + Uo.w; frame_vel(Uo, nx, ny, eps, qu[2], qu[3]);
    }
    T out[4];
    bool done = false;
    if (LIM == kLearned) {
        if (phi >= 0.0f && phi <= 1.0f) {  // a NaN fails both tests
            const T p = T(phi);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const T sb = (qc[i] - qu[i]) * dist.x, sf = (qk[i] - qc[i]) * dist.y;
                out[i] = qc[i] + dm * tvd_clip(p * ((qk[i] - qu[i]) * dist.z), sb, sf);
            }
            done = out[0] >= T(0);
        }
    }
    if (!done) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T sb = (qc[i] - qu[i]) * dist.x, sf = (qk[i] - qc[i]) * dist.y;
            out[i] = qc[i] + dm * limit<T, (LIM == kLearned ? kMinmod : LIM)>(sb, sf);
        }
    }
    if (out[0] < T(0)) return r;
    r.h = out[0];
    r.b = out[1] - out[0];
    r.eta = out[1];
    r.un = out[2];
    r.ut = out[3];
    return r;
}

// HLL wave fan (Sec. 6.2.1): speeds, physical fluxes and star flux; states
// in the normal frame (h, q_n, q_t).  Dry sides use the dry-bed speeds.
template <typename T> struct Fan {
    T hL, hR, uL, uR, vL, vR, qL, qR;
    T GL[3], GR[3], Fs[2];
    T SL, SR, Ss;
    bool dry;
};

template <typename T>
__device__ __forceinline__ void wave_fan(T g, T eps, const T UL[3], const T UR[3], Fan<T> &W)
{
    W.hL = UL[0]; W.hR = UR[0];
    W.dry = (W.hL <= eps && W.hR <= eps);
    const bool wl = W.hL > eps, wr = W.hR > eps;
    W.uL = wl ? fdiv(UL[1], W.hL) : T(0); W.vL = wl ? fdiv(UL[2], W.hL) : T(0);
    W.uR = wr ? fdiv(UR[1], W.hR) : T(0); W.vR = wr ? fdiv(UR[2], W.hR) : T(0);
    W.qL = wl ? UL[1] : T(0); W.qR = wr ? UR[1] : T(0);
    if (W.dry) return;
    const T hL = W.hL, hR = W.hR, uL = W.uL, uR = W.uR;
    const T aL = sqrt(g * hL), aR = sqrt(g * hR);
    if (!wr) {
        W.SL = uL - aL; W.SR = uL + T(2) * aL; W.Ss = W.SR;
    } else if (!wl) {
        W.SL = uR - T(2) * aR; W.SR = uR + aR; W.Ss = W.SL;
    } else {
        const T h0 = T(0.5) * (hL + hR) - fdiv(T(0.25) * (uR - uL) * (hL + hR), aR + aL);
        T hs;
        if (h0 <= tmin(hL, hR)) {
            const T t = T(0.5) * (aR + aL) + T(0.25) * (uL - uR);
            hs = t > T(0) ? fdiv(t * t, g) : T(0);
        } else {
            const T gL = sqrt(fdiv(g * (h0 + hL), T(2) * h0 * hL));
            const T gR = sqrt(fdiv(g * (h0 + hR), T(2) * h0 * hR));
            hs = fdiv(hL * gL + hR * gR + uL - uR, gL + gR);
        }
        const T pL = hs > hL ? sqrt(fdiv((hs + hL) * hs, T(2) * hL * hL)) : T(1);
        const T pR = hs > hR ? sqrt(fdiv((hs + hR) * hs, T(2) * hR * hR)) : T(1);
        W.SL = uL - aL * pL;
        W.SR = uR + aR * pR;
        W.Ss = fdiv(W.SL * hR * (uR - W.SR) - W.SR * hL * (uL - W.SL),
                    hR * (uR - W.SR) - hL * (uL - W.SL));
    }
    W.GL[0] = W.qL; W.GL[1] = W.qL * uL + T(0.5) * g * hL * hL; W.GL[2] = W.qL * W.vL;
    W.GR[0] = W.qR; W.GR[1] = W.qR * uR + T(0.5) * g * hR * hR; W.GR[2] = W.qR * W.vR;
    const T d = W.SR - W.SL;
    W.Fs[0] = fdiv(W.SR * W.GL[0] - W.SL * W.GR[0] + W.SR * W.SL * (hR - hL), d);
    W.Fs[1] = fdiv(W.SR * W.GL[1] - W.SL * W.GR[1] + W.SR * W.SL * (W.qR - W.qL), d);
}

template <typename T>
__device__ __forceinline__ void flux_hllc(T g, T eps, const T UL[3], const T UR[3], T F[3])
{
    Fan<T> W;
    wave_fan(g, eps, UL, UR, W);
    if (W.dry) { F[0] = F[1] = F[2] = T(0); return; }
    if (W.SL >= T(0)) { F[0] = W.GL[0]; F[1] = W.GL[1]; F[2] = W.GL[2]; return; }
    if (W.SR <= T(0)) { F[0] = W.GR[0]; F[1] = W.GR[1]; F[2] = W.GR[2]; return; }
    F[0] = W.Fs[0];
    F[1] = W.Fs[1];
    F[2] = F[0] * (W.Ss >= T(0) ? W.vL : W.vR);  // contact: upwind tangential velocity
}

// WAF (Sec. 6.2.2) with the superbee A(r, c) of eq. (eq:superbee).
template <typename T> __device__ __forceinline__ T superbee_A(T r, T c)
{
    const T ac = c < T(0) ? -c : c;
    if (r <= T(0)) return T(1);
    if (r <= T(0.5)) return T(1) - T(2) * (T(1) - ac) * r;
    if (r <= T(1)) return ac;
    if (r <= T(2)) return T(1) - (T(1) - ac) * r;
    return T(2) * ac - T(1);
}

template <typename T> __device__ __forceinline__ T sgn(T x)
{
    return x > T(0) ? T(1) : (x < T(0) ? T(-1) : T(0));
}

struct WafRatio { bool hasLu, hasRu; };

template <typename T>
__device__ __forceinline__ T waf_ratio(T S, T qL, T qR, T qLu, T qRu, bool hasLu, bool hasRu)
{
    const T dloc = qR - qL;
    if (dloc == T(0)) return T(0);
    if (S >= T(0)) return hasLu ? fdiv(qL - qLu, dloc) : T(0);
    return hasRu ? fdiv(qRu - qR, dloc) : T(0);
}

template <typename T, int MODE> __device__ __forceinline__ T waf_A(T r, T c)
{
    if (MODE == kWafGodunov) return T(1);
    if (MODE == kWafUnlimited) return c < T(0) ? -c : c;
    return superbee_A(r, c);
}

// eta and v of L, R and of their upwind means; has*u: an upwind value exists
template <typename T> struct WafIn {
    T eL, eR, eLu, eRu, vL, vR, vLu, vRu;
    bool hasLu, hasRu;
};

// WAF flux of Sec. 6.2.2 (TVD weights with the superbee A of eq.
// eq:superbee, or the Godunov / unlimited weights).
template <typename T, int MODE>
__device__ __forceinline__ void flux_waf(T g, T eps, T dt_dx, const T UL[3], const T UR[3],
                                         const WafIn<T> &w, T F[3])
{
    Fan<T> W;
    wave_fan(g, eps, UL, UR, W);
    if (W.dry) { F[0] = F[1] = F[2] = T(0); return; }
    const T cL = W.SL * dt_dx, cR = W.SR * dt_dx, cs = W.Ss * dt_dx;
    const T AL = waf_A<T, MODE>(waf_ratio(W.SL, w.eL, w.eR, w.eLu, w.eRu, w.hasLu, w.hasRu), cL);
    const T AR = waf_A<T, MODE>(waf_ratio(W.SR, w.eL, w.eR, w.eLu, w.eRu, w.hasLu, w.hasRu), cR);
    const T As = waf_A<T, MODE>(waf_ratio(W.Ss, w.vL, w.vR, w.vLu, w.vRu, w.hasLu, w.hasRu), cs);
    const T wL = T(0.5) * (T(1) + sgn(cL) * AL);
    const T wLR = T(0.5) * (sgn(cR) * AR - sgn(cL) * AL);
    const T wR = T(0.5) * (T(1) - sgn(cR) * AR);
#pragma unroll
    for (int i = 0; i < 2; ++i) F[i] = wL * W.GL[i] + wLR * W.Fs[i] + wR * W.GR[i];
    const T wLs = T(0.5) * (T(1) + sgn(cs) * As), wRs = T(0.5) * (T(1) - sgn(cs) * As);
    F[2] = (wLs * W.vL + wRs * W.vR) * F[0];
}

// Positivity of WAF's depths.  Over one step an edge may take from the
// cell it drains at most the share L / P of that cell's water (L the edge
// length, P the perimeter): a mass flux of at most h |Omega| / (P dt) =
// h R / (2 dt), R = 2 |Omega| / P the inscribed radius, so that summed over
// its three edges no cell loses more than it holds; the bound is taken at
// 99% of the share so that rounding cannot take the last drop.  A WAF flux
// whose mass component leaves the bounds of L (flux from L to R) or R (the
// reverse) is blended towards the first-order HLLC flux of the same states,
// F = F_hllc + theta (F_waf - F_hllc), with the largest theta in [0, 1]
// meeting the bound, and its mass component is set to the bound; when HLLC
// is itself beyond the bound the edge takes HLLC.  hL, hR: the cells'
// depths; RL, RR: their inscribed radii (canonical orientation, so both
// sides of an edge compute the same bits).
template <typename T>
__device__ __forceinline__ void waf_positivity(T g, T eps, const T UL[3], const T UR[3], T hL, T RL,
                                               T hR, T RR, T dt, T F[3])
{
    const T hi = fdiv(T(0.99) * hL * RL, T(2) * dt), lo = -fdiv(T(0.99) * hR * RR, T(2) * dt);
    if (F[0] <= hi && F[0] >= lo) return;
    const T bound = F[0] > hi ? hi : lo;
    T Fh[3];
    flux_hllc(g, eps, UL, UR, Fh);
    const T theta = fdiv(bound - Fh[0], F[0] - Fh[0]);
    if (!(theta > T(0))) {
        F[0] = Fh[0]; F[1] = Fh[1]; F[2] = Fh[2];
    } else if (theta < T(1)) {
        F[1] = Fh[1] + theta * (F[1] - Fh[1]);
        F[2] = Fh[2] + theta * (F[2] - Fh[2]);
        F[0] = bound;
    }
}

}  // namespace swe

namespace swe {

// tanh for the limiter features: exact in FP64; in FP32 through one hardware
// exp2 and one reciprocal (about 1e-6 absolute, far below the BF16 rounding
// the features then get).
template <typename T> __device__ __forceinline__ T ftanh(T x) { return tanh(x); }
template <> __device__ __forceinline__ float ftanh<float>(float x)
{
    const float xc = fminf(fmaxf(x, -15.0f), 15.0f);
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * xc);  // exp(2x)
    return (e - 1.0f) * __builtin_amdgcn_rcpf(e + 1.0f);
}

constexpr int kMlpIn = 14, kMlpH = 32;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;  // 1569

// Inputs of the learned limiter for the half-edge of cell c across local
// edge m (a design of this library; the paper has no learned limiter): for
// h, q_n, q_t (discharges in the edge frame) and b, the upwind and
// cross-edge increments to the edge midpoint ab = sb d_mid and af = sf d_mid
// as tanh(a / scale) (for q_t, whose sign flips in a mirror image, of |a|:
// the features of mirror-image half-edges are equal) and their ratio
// ab af / (af^2 + (0.01 scale)^2) clipped to
// [-2, 2]; then tanh of the cell's Froude
// number and of the relative depth jump across the edge.  Scales: h, b:
// h_c + 0.01 m; q: h_c sqrt(g h_c) + 0.01 m^2/s.  Returns false when the
// half-edge is not reconstructed to second order (dry stencil cell, no
// neighbour across the edge, no upwind cell): the features are then zero.
template <typename T, typename T4>
__device__ __forceinline__ bool limiter_features(const T4 &Uc, const T4 &Uk, bool hk_, const T4 &Ua,
                                                 bool ha, const T4 &Ub, bool hb, T nx, T ny, T al,
                                                 T be, T g, T eps, float f[kMlpIn])
{
    // one test up front (a wave whose half-edges are all dry or one-sided
    // skips the rest), then no divergent branch: the upwind state is a select
    const bool ok = hk_ && Uc.x > eps && Uk.x > eps && (!ha || Ua.x > eps) && (!hb || Ub.x > eps) &&
                    (ha || hb);
    if (!ok) {
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) f[i] = 0.0f;
        return false;
    }
    const T qc[4] = {Uc.x, Uc.y * nx + Uc.z * ny, -Uc.y * ny + Uc.z * nx, Uc.w};
    const T qk[4] = {Uk.x, Uk.y * nx + Uk.z * ny, -Uk.y * ny + Uk.z * nx, Uk.w};
    // upwind state: the mean of the two upwind cells, or the one that exists
    const bool both = ha && hb;
    const T4 &Uo = ha ? Ua : Ub;
    T qu[4];
    qu[0] = both ? T(0.5) * (Ua.x + Ub.x) : Uo.x;
    qu[1] = both ? T(0.5) * ((Ua.y * nx + Ua.z * ny) + (Ub.y * nx + Ub.z * ny)) : Uo.y * nx + Uo.z * ny;
    qu[2] = both ? T(0.5) * ((-Ua.y * ny + Ua.z * nx) + (-Ub.y * ny + Ub.z * nx))
                 : -Uo.y * ny + Uo.z * nx;
    qu[3] = both ? T(0.5) * (Ua.w + Ub.w) : Uo.w;
    const T hc = Uc.x;
    const T sh = hc + T(0.01), sq = hc * sqrt(g * hc) + T(0.01);
    const T sc[4] = {sh, sq, sq, sh};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // upwind and cross-edge increments over the distance to the edge
        // midpoint (slope times d_mid): the MUSCL weights al = d_mid / d_up
        // and be = d_mid / d_fwd times the differences
        const T ab = al * (qc[k] - qu[k]), af = be * (qk[k] - qc[k]);
        const T isc = frcp(sc[k]);
        // q_t changes sign in a mirror image: its increments enter by
        // magnitude (the ratio keeps their relative sign)
        f[3 * k + 0] = float(ftanh((k == 2 ? fabs(ab) : ab) * isc));
        f[3 * k + 1] = float(ftanh((k == 2 ? fabs(af) : af) * isc));
        // regularized at 1% of the scale: smooth where af vanishes
        const T r = fdiv(ab * af, af * af + T(1e-4) * sc[k] * sc[k]);
        f[3 * k + 2] = float(tmin(T(2), tmax(T(-2), r)));
    }
    const T ih = frcp(hc);
    const T uc = Uc.y * ih, vc = Uc.z * ih;
    const T un = uc * nx + vc * ny, ut = -uc * ny + vc * nx;
    f[12] = float(ftanh(fdiv(sqrt(un * un + ut * ut), sqrt(g * tmax(hc, T(1e-6))))));
    f[13] = float(ftanh(fdiv(Uk.x - hc, hc + T(0.01))));
    return true;
}

}  // namespace swe

// ------------------------------------------------------------------------
// Primitive-variable forms used by the tiled stage kernel: velocities are
// formed once per cell (u = hu/h, zero where dry) and the Riemann solver
// takes (h, u_n, u_t) directly, so no discharge is divided by a depth twice.
// FP32 uses the hardware reciprocal (1 ulp); FP64 divides exactly.
namespace swe {


template <typename T> struct Prim { T h, b, u, v; };

template <typename T, typename T4>
__device__ __forceinline__ Prim<T> prim(const T4 &U, T eps)
{
    Prim<T> p;
    p.h = U.x;
    p.b = U.w;
    const T r = U.x > eps ? frcp(U.x) : T(0);
    p.u = U.y * r;
    p.v = U.z * r;
    return p;
}

// beta limiters in branch-free form: zero unless both slopes have the same
// sign (their product is positive), else the signed
// max(min(beta|sb|, |sf|), min(|sb|, beta|sf|)); this is the printed
// MINBEE/SUPERBEE form of Sec. 6.2.3 value for value (but for slopes whose
// product underflows, which count as zero).
template <typename T, int LIM>
__device__ __forceinline__ T limit2(T sb, T sf)
{
    if (LIM == kZeroSlope) return T(0);
    if constexpr (sizeof(T) == 4 && (LIM == kMinmod || LIM == kSuperbee)) {
        // the same values by median selections (exact): minmod(a, b) is the
        // median of a, b and 0; superbee is the larger in magnitude of
        // minmod(2 sb, sf) and minmod(sb, 2 sf).  (Slopes whose product
        // underflows keep their minmod value here instead of counting as zero.)
        if (LIM == kMinmod) return __builtin_amdgcn_fmed3f(sb, sf, 0.0f);
        const float s1 = __builtin_amdgcn_fmed3f(2.0f * sb, sf, 0.0f);
        const float s2 = __builtin_amdgcn_fmed3f(sb, 2.0f * sf, 0.0f);
        return sf > 0.0f ? fmaxf(s1, s2) : fminf(s1, s2);
    }
    const T p = sb * sf;
    // a true quotient: with FP64 denormals sb^2 + sf^2 can be far below
    // 1 / DBL_MAX, where a reciprocal overflows and 0 * inf would give NaN
    if (LIM == kVanAlbada) return p > T(0) ? fdiv(p * (sb + sf), sb * sb + sf * sf) : T(0);
    const T ab = fabs(sb), af = fabs(sf);
    const T m = LIM == kSuperbee ? tmax(tmin(T(2) * ab, af), tmin(ab, T(2) * af)) : tmin(ab, af);
    return p > T(0) ? copysign(m, sf) : T(0);
}

// Interface values of cell C across an interior edge with outward normal n
// (Sec. 6.2.3 on the rotated states), K across the edge, A and B the upwind
// cells, with the distances folded into weights: al = d_mid / d_up and
// be = d_mid / d_fwd for the limited slope, ga = d_mid / d_central for the
// learned limiter's scaled central slope.
template <typename T, bool MUSCL_, int LIM>
__device__ __forceinline__ Half<T> recon3(const Prim<T> &C, const Prim<T> &K, const Prim<T> &A,
                                          bool ha, const Prim<T> &B, bool hb, T nx, T ny, T al,
                                          T be, T ga, float phi, T eps)
{
    Half<T> r;
    r.h = C.h;
    r.b = C.b;
    r.eta = C.h + C.b;
    r.un = C.u * nx + C.v * ny;
    r.ut = -C.u * ny + C.v * nx;
    if (!MUSCL_) return r;
    if (!(C.h > eps) || !(K.h > eps)) return r;
    if ((ha && !(A.h > eps)) || (hb && !(B.h > eps)) || (!ha && !hb)) return r;
    const T qc[4] = {C.h, C.h + C.b, r.un, r.ut};
    const T qk[4] = {K.h, K.h + K.b, K.u * nx + K.v * ny, -K.u * ny + K.v * nx};
    // upwind state: the mean of the upwind cells (rotation is linear, so the
    // mean velocity is rotated once), or the one that exists
    const bool both = ha && hb;
    const Prim<T> &O = ha ? A : B;
    const T uh = both ? T(0.5) * (A.h + B.h) : O.h;
    const T ue = both ? T(0.5) * ((A.h + A.b) + (B.h + B.b)) : O.h + O.b;
    const T uu = both ? T(0.5) * (A.u + B.u) : O.u;
    const T uv = both ? T(0.5) * (A.v + B.v) : O.v;
    const T qu[4] = {uh, ue, uu * nx + uv * ny, -uu * ny + uv * nx};
    T out[4];
    bool done = false;
    if (LIM == kLearned) {
        if (phi >= 0.0f && phi <= 1.0f) {
            const T p = T(phi);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[i] = qc[i] + tvd_clip(p * (ga * (qk[i] - qu[i])), al * (qc[i] - qu[i]),
                                          be * (qk[i] - qc[i]));
            done = out[0] >= T(0);
        }
    }
    if (!done) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            out[i] = qc[i] + limit2<T, (LIM == kLearned ? kMinmod : LIM)>(al * (qc[i] - qu[i]),
                                                                          be * (qk[i] - qc[i]));
    }
    if (out[0] < T(0)) return r;
    r.h = out[0];
    r.b = out[1] - out[0];
    r.eta = out[1];
    r.un = out[2];
    r.ut = out[3];
    return r;
}

// HLLC of Sec. 6.2.1 from depths and normal-frame velocities (the same
// estimates as wave_fan / flux_hllc).
template <typename T>
__device__ __forceinline__ void hllc_prim(T g, T eps, T hL, T uL, T vL, T hR, T uR, T vR, T F[3])
{
    const bool wl = hL > eps, wr = hR > eps;
    if (!wl && !wr) { F[0] = F[1] = F[2] = T(0); return; }
    if (!wl) { uL = T(0); vL = T(0); }
    if (!wr) { uR = T(0); vR = T(0); }
    const T qL = wl ? hL * uL : T(0), qR = wr ? hR * uR : T(0);
    const T aL = sqrt(g * hL), aR = sqrt(g * hR);
    T SL, SR, Ss;
    if (!wr) {
        SL = uL - aL; SR = uL + T(2) * aL; Ss = SR;
    } else if (!wl) {
        SL = uR - T(2) * aR; SR = uR + aR; Ss = SL;
    } else {
        const T h0 = T(0.5) * (hL + hR) - T(0.25) * (uR - uL) * (hL + hR) * frcp(aR + aL);
        T hs;
        if (h0 <= tmin(hL, hR)) {
            const T t = T(0.5) * (aR + aL) + T(0.25) * (uL - uR);
            hs = t > T(0) ? t * t * frcp(g) : T(0);
        } else {
            const T gL = sqrt(g * (h0 + hL) * frcp(T(2) * h0 * hL));
            const T gR = sqrt(g * (h0 + hR) * frcp(T(2) * h0 * hR));
            hs = (hL * gL + hR * gR + uL - uR) * frcp(gL + gR);
        }
        const T pL = hs > hL ? sqrt((hs + hL) * hs * frcp(T(2) * hL * hL)) : T(1);
        const T pR = hs > hR ? sqrt((hs + hR) * hs * frcp(T(2) * hR * hR)) : T(1);
        SL = uL - aL * pL;
        SR = uR + aR * pR;
        Ss = (SL * hR * (uR - SR) - SR * hL * (uL - SL)) * frcp(hR * (uR - SR) - hL * (uL - SL));
    }
    const T GL1 = qL * uL + T(0.5) * g * hL * hL, GR1 = qR * uR + T(0.5) * g * hR * hR;
    if (SL >= T(0)) { F[0] = qL; F[1] = GL1; F[2] = qL * vL; return; }
    if (SR <= T(0)) { F[0] = qR; F[1] = GR1; F[2] = qR * vR; return; }
    const T inv = frcp(SR - SL);
    F[0] = (SR * qL - SL * qR + SR * SL * (hR - hL)) * inv;
    F[1] = (SR * GL1 - SL * GR1 + SR * SL * (qR - qL)) * inv;
    F[2] = F[0] * (Ss >= T(0) ? vL : vR);
}

// HLLC of Sec. 6.2.1 (the estimates of hllc_prim) in pressure-deviation
// form: the mass flux F0, the tangential flux F2 and, for the normal
// momentum, the flux less either side's hydrostatic pressure,
// DL = F1 - g hL^2 / 2 and DR = F1 - g hR^2 / 2.  The pressure difference
// enters as g (hL - hR)(hL + hR) / 2, so a state at rest (zero velocities,
// equal depths) gives exactly zero in any precision.
template <typename T>
__device__ __forceinline__ void hllc_dev(T g, T eps, T hL, T uL, T vL, T hR, T uR, T vR, T &F0,
                                         T &DL, T &DR, T &F2)
{
    const bool wl = hL > eps, wr = hR > eps;
    if (!wl && !wr) {
        F0 = T(0); F2 = T(0);
        DL = -(T(0.5) * g * hL * hL);
        DR = -(T(0.5) * g * hR * hR);
        return;
    }
    if (!wl) { uL = T(0); vL = T(0); }
    if (!wr) { uR = T(0); vR = T(0); }
    const T qL = wl ? hL * uL : T(0), qR = wr ? hR * uR : T(0);
    const T aL = sqrt(g * hL), aR = sqrt(g * hR);
    T SL, SR, Ss;
    if (!wr) {
        SL = uL - aL; SR = uL + T(2) * aL; Ss = SR;
    } else if (!wl) {
        SL = uR - T(2) * aR; SR = uR + aR; Ss = SL;
    } else {
        const T h0 = T(0.5) * (hL + hR) - T(0.25) * (uR - uL) * (hL + hR) * frcp(aR + aL);
        T hs;
        if (h0 <= tmin(hL, hR)) {
            const T t = T(0.5) * (aR + aL) + T(0.25) * (uL - uR);
            hs = t > T(0) ? t * t * frcp(g) : T(0);
        } else {
            const T gL = sqrt(g * (h0 + hL) * frcp(T(2) * h0 * hL));
            const T gR = sqrt(g * (h0 + hR) * frcp(T(2) * h0 * hR));
            hs = (hL * gL + hR * gR + uL - uR) * frcp(gL + gR);
        }
        const T pL = hs > hL ? sqrt((hs + hL) * hs * frcp(T(2) * hL * hL)) : T(1);
        const T pR = hs > hR ? sqrt((hs + hR) * hs * frcp(T(2) * hR * hR)) : T(1);
        SL = uL - aL * pL;
        SR = uR + aR * pR;
        Ss = (SL * hR * (uR - SR) - SR * hL * (uL - SL)) * frcp(hR * (uR - SR) - hL * (uL - SL));
    }
    const T dP = T(0.5) * g * (hL - hR) * (hL + hR);  // pL - pR
    const T mL = qL * uL, mR = qR * uR;                // advective momentum fluxes
    if (SL >= T(0)) { F0 = qL; DL = mL; DR = mL + dP; F2 = qL * vL; return; }
    if (SR <= T(0)) { F0 = qR; DL = mR - dP; DR = mR; F2 = qR * vR; return; }
    const T inv = frcp(SR - SL);
    F0 = (SR * qL - SL * qR + SR * SL * (hR - hL)) * inv;
    const T base = SR * mL - SL * mR + SR * SL * (qR - qL);
    DL = (base + SL * dP) * inv;
    DR = (base + SR * dP) * inv;
    F2 = F0 * (Ss >= T(0) ? vL : vR);
}

// A cell's share of an edge (Sec. 6.1): the oriented flux sg * G plus the
// side correction p along the cell's own normal, as explicit fused
// multiply-adds so that both cells of an edge, and both places an edge can
// be evaluated, round identically.
template <typename T>
__device__ __forceinline__ void half_edge_flux(T sg, T G0, T G1, T G2, T p, T nx, T ny, T &f0,
                                               T &f1, T &f2)
{
    f0 = sg * G0;
    f1 = fma(p, nx, sg * G1);
    f2 = fma(p, ny, sg * G2);
}

}  // namespace swe
