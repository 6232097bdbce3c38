// Learned slope limiter of libswe.so (an addition of this library, not part
// of the paper's method): a per-half-edge network 14 -> 32 -> 32 -> 1 (ReLU,
// ReLU, sigmoid) whose output phi in [0, 1] scales the central MUSCL slope
// (U_R - U_Lupw)/|x_R - x_Lupw| of Sec. 6.2.3.
//
//  * Inference (swe_mlp_dev.h): BF16 weights and activations on the matrix
//    cores, FP32 accumulation, 64 half-edges per wave in four tiles of 16
//    (five MFMAs per tile: two v_mfma_f32_16x16x16bf16_1k for the
//    14-input layer, v_mfma_f32_16x16x32_bf16 for the hidden and the output
//    layer).  k_limiter_phi evaluates every half-edge of the mesh ahead of
//    a step (one thread per cell builds the features of its three
//    half-edges); the tiled stage kernel can evaluate the same network
//    inside its first phase instead (phi_in_stage).
//  * Training data (k_restrict, k_pairs): the fine-mesh state restricted to
//    the coarse mesh (mean of the four red-refinement children) gives the
//    stencils; the target of a half-edge is the mean of the two children of
//    the coarse cell that touch that edge.
//  * Training (k_train_partial, k_train_reduce, k_adam): FP32 forward and
//    backward, per-block gradient partials reduced in a fixed order
//    (deterministic), Adam on FP32 master weights, BF16 copies for inference.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "swe_ctx.h"
#include "swe_internal.h"
#include "swe_kernels.h"
#include "swe_mlp_dev.h"

using namespace swe;

namespace {

constexpr int kRec = 40;  // floats per training record

__device__ __forceinline__ int xcd_tile_m(int bid, int nb)
{
    const int x = bid & 7, i = bid >> 3, base = nb >> 3, rem = nb & 7;
    return x * base + (x < rem ? x : rem) + i;
}

void pack_mlp(const float *p, MlpDev &w)
{
    std::memset(&w, 0, sizeof(w));
    const float *W1 = p, *b1 = p + kMlpH * kMlpIn, *W2 = b1 + kMlpH, *b2 = W2 + kMlpH * kMlpH;
    const float *W3 = b2 + kMlpH, *b3 = W3 + kMlpH;
    for (int j = 0; j < kMlpH; ++j) {
        for (int i = 0; i < kMlpIn; ++i) w.W1[j * 16 + i] = bf16_bits(W1[j * kMlpIn + i]);
        for (int i = 0; i < kMlpH; ++i) w.W2[j * kMlpH + i] = bf16_bits(W2[j * kMlpH + i]);
        w.b1[j] = bf16_float(bf16_bits(b1[j]));
        w.b2[j] = bf16_float(bf16_bits(b2[j]));
        w.W3[j] = bf16_float(bf16_bits(W3[j]));
    }
    w.b3 = bf16_float(bf16_bits(b3[0]));
}

template <typename T> struct PhiArgs {
    using T4 = typename V4<T>::type;
    int n;
    const int4 *nbr;
    const T4 *he_co, *U;  // he_co: nx, ny, d_mid / d_up, d_mid / d_fwd per half-edge (edge-major)
    const MlpDev *w;
    float *phi;
    T g, eps;
};

template <typename T>
__global__ void __launch_bounds__(256) k_limiter_phi(PhiArgs<T> a)
{
    using T4 = typename V4<T>::type;
    __shared__ __align__(16) uint16_t X[4][192][16];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c0 = xcd_tile_m(blockIdx.x, gridDim.x) * 256 + wv * 64;
    const int c = c0 + lane;
    if (c < a.n) {
        const int4 nb4 = a.nbr[c];
        const T4 Uc = a.U[c];
        // neighbours in separate variables, picked by selects (a local array
        // indexed at run time would live in scratch memory)
        const bool hn0 = nb4.x >= 0, hn1 = nb4.y >= 0, hn2 = nb4.z >= 0;
        // (the index is selected, not the value: a select between a load and
        // a local value becomes a load through a selected pointer, which
        // puts the local value in scratch memory)
        const T4 Un0 = a.U[hn0 ? nb4.x : c], Un1 = a.U[hn1 ? nb4.y : c], Un2 = a.U[hn2 ? nb4.z : c];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int ma = (m + 1) % 3, mb = (m + 2) % 3;
            const T4 Um = m == 0 ? Un0 : (m == 1 ? Un1 : Un2);
            const T4 Ua = ma == 0 ? Un0 : (ma == 1 ? Un1 : Un2);
            const T4 Ub = mb == 0 ? Un0 : (mb == 1 ? Un1 : Un2);
            const bool hm = m == 0 ? hn0 : (m == 1 ? hn1 : hn2);
            const bool ha = ma == 0 ? hn0 : (ma == 1 ? hn1 : hn2);
            const bool hb = mb == 0 ? hn0 : (mb == 1 ? hn1 : hn2);
            float f[kMlpIn];
            const T4 co = a.he_co[m * a.n + c];
            const bool ok = limiter_features<T, T4>(Uc, Um, hm, Ua, ha, Ub, hb, co.x, co.y, co.z,
                                                    co.w, a.g, a.eps, f);
            mlp_write_row(X[wv][3 * lane + m], f, ok);
        }
    } else {
        const float f0[kMlpIn] = {};
#pragma unroll
        for (int m = 0; m < 3; ++m) mlp_write_row(X[wv][3 * lane + m], f0, false);
    }
    const MlpLane L = mlp_lane(a.w, lane);
    wave_lds_sync();
    // rows 3 l + m (cell l of the wave, local edge m) in three groups of 64
    for (int rg = 0; rg < 3; ++rg) {
        const int row = rg * 64 + lane;
        const float z = mlp_rows_z(L, X[wv] + rg * 64, lane);
        const float ph = mlp_phi(z, X[wv][row][15] != 0);
        if (c0 + row / 3 < a.n) a.phi[3 * c0 + row] = ph;
    }
}

// ----------------------------------------------------------- training data
template <typename T>
__global__ void k_restrict(int n, const int *children, int n_fine, const typename V4<T>::type *Uf,
                           const T *bed, typename V4<T>::type *Uc, int *bad)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int k = 0; k < 4; ++k)
        if (children[4 * c + k] < 0 || children[4 * c + k] >= n_fine) { atomicOr(bad, 1); return; }
    typename V4<T>::type s;
    s.w = bed[c];
    T h = 0, hu = 0, hv = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const typename V4<T>::type u = Uf[children[4 * c + k]];
        h += u.x; hu += u.y; hv += u.z;
    }
    s.x = T(0.25) * h; s.y = T(0.25) * hu; s.z = T(0.25) * hv;
    Uc[c] = s;  // the bed stays the coarse cell's
}

template <typename T> struct PairArgs {
    using T4 = typename V4<T>::type;
    int n;
    const int4 *nbr;
    const T4 *he_geo, *he_dist, *he_co, *U, *Uf;
    const int *children;
    int n_fine;
    float *rec;
    T g, eps;
};

// One record per coarse half-edge: features[14], q[4] = (h, eta, u_n, u_t) of
// the cell, s[4] central slopes, target distance d_mid / 2, target[4], valid.
template <typename T>
__global__ void k_pairs(PairArgs<T> a)
{
    using T4 = typename V4<T>::type;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const int4 nb4 = a.nbr[c];
    const int nb[3] = {nb4.x, nb4.y, nb4.z};
    const T4 Uc = a.U[c];
    T4 Un[3];
    bool hn[3];
    for (int m = 0; m < 3; ++m) {
        hn[m] = nb[m] >= 0;
        Un[m] = hn[m] ? a.U[nb[m]] : Uc;
    }
    const T eps = a.eps;
    for (int m = 0; m < 3; ++m) {
        float *r = a.rec + (size_t)kRec * (3 * c + m);
        const int ma = (m + 1) % 3, mb = (m + 2) % 3;
        const T4 ge = a.he_geo[3 * c + m];
        const T4 di = a.he_dist[3 * c + m];
        const T nx = ge.x, ny = ge.y;
        float f[kMlpIn];
        const T4 co = a.he_co[m * a.n + c];
        bool ok = limiter_features<T, T4>(Uc, Un[m], hn[m], Un[ma], hn[ma], Un[mb], hn[mb], co.x, co.y,
                                          co.z, co.w, a.g, eps, f);
        for (int i = 0; i < kMlpIn; ++i) r[i] = f[i];
        T qc[4] = {Uc.x, Uc.x + Uc.w, T(0), T(0)};
        frame_vel(Uc, nx, ny, eps, qc[2], qc[3]);
        T s[4] = {0, 0, 0, 0}, sb[4] = {0, 0, 0, 0}, sf[4] = {0, 0, 0, 0};
        if (ok) {
            const T4 &Uk = Un[m];
            T qk[4] = {Uk.x, Uk.x + Uk.w, T(0), T(0)};
            frame_vel(Uk, nx, ny, eps, qk[2], qk[3]);
            T qu[4];
            if (hn[ma] && hn[mb]) {
                T qa[4] = {Un[ma].x, Un[ma].x + Un[ma].w, 0, 0}, qb[4] = {Un[mb].x, Un[mb].x + Un[mb].w, 0, 0};
                frame_vel(Un[ma], nx, ny, eps, qa[2], qa[3]);
                frame_vel(Un[mb], nx, ny, eps, qb[2], qb[3]);
                for (int i = 0; i < 4; ++i) qu[i] = T(0.5) * (qa[i] + qb[i]);
            } else {
                const T4 &Uo = hn[ma] ? Un[ma] : Un[mb];
                qu[0] = Uo.x; qu[1] = Uo.x + Uo.w;
                frame_vel(Uo, nx, ny, eps, qu[2], qu[3]);
            }
            for (int i = 0; i < 4; ++i) {
                s[i] = (qk[i] - qu[i]) * di.z;
                sb[i] = (qc[i] - qu[i]) * di.x;
                sf[i] = (qk[i] - qc[i]) * di.y;
            }
        }
        // target: mean of the two children touching edge m (at parent nodes m, m+1)
        const int ia = a.children[4 * c + m], ib = a.children[4 * c + (m + 1) % 3];
        for (int i = 0; i < 4; ++i) { r[32 + i] = float(sb[i]); r[36 + i] = float(sf[i]); }
        if (ia < 0 || ia >= a.n_fine || ib < 0 || ib >= a.n_fine) { r[27] = 0.0f; continue; }
        const T4 fa = a.Uf[ia], fb = a.Uf[ib];
        T ua, va, ub, vb;
        frame_vel(fa, nx, ny, eps, ua, va);
        frame_vel(fb, nx, ny, eps, ub, vb);
        const bool wet = fa.x > eps && fb.x > eps;
        for (int i = 0; i < 4; ++i) { r[14 + i] = float(qc[i]); r[18 + i] = float(s[i]); }
        // the two children touching edge m have their mean centroid halfway
        // between the coarse centroid and the edge midpoint (red refinement:
        // (5A + 5B + 2C) / 12 against (A + B + C) / 3 and (A + B) / 2), so
        // the target is the fine solution at distance d_mid / 2
        r[22] = float(T(0.5) * ge.w);
        r[23] = float(T(0.5) * (fa.x + fb.x));
        r[24] = float(T(0.5) * ((fa.x + fa.w) + (fb.x + fb.w)));
        r[25] = float(T(0.5) * (ua + ub));
        r[26] = float(T(0.5) * (va + vb));
        r[27] = (ok && wet) ? 1.0f : 0.0f;
        // the classic (minmod) interface values of the same half-edge, for
        // comparing the two limiters against the same targets
        const Half<T> mm = reconstruct<T, T4, kMUSCL, kMinmod>(Uc, Un[m], Un[ma], hn[ma], Un[mb], hn[mb],
                                                               nx, ny, ge.w, di, 0.0f, eps);
        r[28] = float(mm.h);
        r[29] = float(mm.h + mm.b);
        r[30] = float(mm.un);
        r[31] = float(mm.ut);
    }
}

// -------------------------------------------------------------- training
constexpr int kChunk = 64;

struct TrainArgs {
    const float *rec;
    const int *idx;
    int n, n_rec;
    const float *params;   // FP32 masters [1569]
    float wv[4];
    float *partial;        // [gridDim.x][kMlpParams + 1]
};

__global__ void __launch_bounds__(256) k_train_partial(TrainArgs a)
{
    __shared__ float P[kMlpParams];
    __shared__ float sx[kChunk][kMlpIn], sa1[kChunk][kMlpH], sa2[kChunk][kMlpH];
    __shared__ float sd1[kChunk][kMlpH], sd2[kChunk][kMlpH], sdz[kChunk], sloss[kChunk];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) P[i] = a.params[i];
    const float *W1 = P, *b1 = P + kMlpH * kMlpIn, *W2 = b1 + kMlpH, *b2 = W2 + kMlpH * kMlpH;
    const float *W3 = b2 + kMlpH, *b3 = W3 + kMlpH;
    constexpr int kSlots = (kMlpParams + 255) / 256;
    float acc[kSlots];
    for (int i = 0; i < kSlots; ++i) acc[i] = 0.f;
    float lacc = 0.f;
    __syncthreads();
    const int nchunks = (a.n + kChunk - 1) / kChunk;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int t = threadIdx.x;
        if (t < kChunk) {
            const int si = ch * kChunk + t;
            float a1[kMlpH], a2[kMlpH];
            const int ri = si < a.n ? a.idx[si] : -1;
            if (ri >= 0 && ri < a.n_rec) {
                const float *r = a.rec + (size_t)kRec * ri;
                float x[kMlpIn];
                for (int i = 0; i < kMlpIn; ++i) { x[i] = r[i]; sx[t][i] = x[i]; }
                for (int j = 0; j < kMlpH; ++j) {
                    float s = b1[j];
                    for (int i = 0; i < kMlpIn; ++i) s += W1[j * kMlpIn + i] * x[i];
                    a1[j] = fmaxf(s, 0.f);
                }
                for (int j = 0; j < kMlpH; ++j) {
                    float s = b2[j];
                    for (int i = 0; i < kMlpH; ++i) s += W2[j * kMlpH + i] * a1[i];
                    a2[j] = fmaxf(s, 0.f);
                }
                float z = b3[0];
                for (int i = 0; i < kMlpH; ++i) z += W3[i] * a2[i];
                const float phi = 1.0f / (1.0f + expf(-z));
                // the value the solver reconstructs with this phi: the
                // scaled central slope kept in the TVD region of the
                // backward and forward slopes (no dependence on phi where
                // the bound or the sign test decides)
                float dphi = 0.f, loss = 0.f;
                for (int k = 0; k < 4; ++k) {
                    const float sc = r[18 + k], sb = r[32 + k], sf = r[36 + k];
                    const float sp = phi * sc;
                    const bool pass = sb * sf > 0.f && fabsf(sp) < 2.f * fminf(fabsf(sb), fabsf(sf));
                    const float cl = sb * sf > 0.f ? copysignf(fminf(fabsf(sp), 2.f * fminf(fabsf(sb), fabsf(sf))), sf)
                                                   : 0.f;
                    const float res = r[14 + k] + r[22] * cl - r[23 + k];
                    loss += a.wv[k] * res * res;
                    if (pass) dphi += 2.0f * a.wv[k] * res * r[22] * copysignf(fabsf(sc), sf);
                }
                const float dz = dphi * phi * (1.0f - phi) / (float)a.n;
                sdz[t] = dz;
                sloss[t] = loss;
                float d2[kMlpH];
                for (int i = 0; i < kMlpH; ++i) d2[i] = a2[i] > 0.f ? dz * W3[i] : 0.f;
                for (int i = 0; i < kMlpH; ++i) {
                    float s = 0.f;
                    for (int j = 0; j < kMlpH; ++j) s += d2[j] * W2[j * kMlpH + i];
                    sd1[t][i] = a1[i] > 0.f ? s : 0.f;
                }
                for (int i = 0; i < kMlpH; ++i) { sa1[t][i] = a1[i]; sa2[t][i] = a2[i]; sd2[t][i] = d2[i]; }
            } else {
                for (int i = 0; i < kMlpIn; ++i) sx[t][i] = 0.f;
                for (int i = 0; i < kMlpH; ++i) { sa1[t][i] = 0.f; sa2[t][i] = 0.f; sd1[t][i] = 0.f; sd2[t][i] = 0.f; }
                sdz[t] = 0.f;
                sloss[t] = 0.f;
            }
        }
        __syncthreads();
        for (int sl = 0; sl < kSlots; ++sl) {
            const int p = threadIdx.x + 256 * sl;
            if (p >= kMlpParams) break;
            float g = 0.f;
            if (p < kMlpH * kMlpIn) {
                const int j = p / kMlpIn, i = p % kMlpIn;
                for (int s = 0; s < kChunk; ++s) g += sd1[s][j] * sx[s][i];
            } else if (p < kMlpH * kMlpIn + kMlpH) {
                const int j = p - kMlpH * kMlpIn;
                for (int s = 0; s < kChunk; ++s) g += sd1[s][j];
            } else if (p < kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH) {
                const int q = p - (kMlpH * kMlpIn + kMlpH), j = q / kMlpH, i = q % kMlpH;
                for (int s = 0; s < kChunk; ++s) g += sd2[s][j] * sa1[s][i];
            } else if (p < kMlpH * kMlpIn + 2 * kMlpH + kMlpH * kMlpH) {
                const int j = p - (kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH);
                for (int s = 0; s < kChunk; ++s) g += sd2[s][j];
            } else if (p < kMlpParams - 1) {
                const int i = p - (kMlpH * kMlpIn + 2 * kMlpH + kMlpH * kMlpH);
                for (int s = 0; s < kChunk; ++s) g += sdz[s] * sa2[s][i];
            } else {
                for (int s = 0; s < kChunk; ++s) g += sdz[s];
            }
            acc[sl] += g;
        }
        if (threadIdx.x == 0)
            for (int s = 0; s < kChunk; ++s) lacc += sloss[s];
        __syncthreads();
    }
    float *out = a.partial + (size_t)blockIdx.x * (kMlpParams + 1);
    for (int sl = 0; sl < kSlots; ++sl) {
        const int p = threadIdx.x + 256 * sl;
        if (p < kMlpParams) out[p] = acc[sl];
    }
    if (threadIdx.x == 0) out[kMlpParams] = lacc;
}

// fixed-order sum of the block partials: grad[p], loss (mean over n)
__global__ void k_train_reduce(const float *partial, int nblocks, int n, float *grad_loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * (kMlpParams + 1) + p];
    grad_loss[p] = p == kMlpParams ? float(s / n) : float(s);
}

__global__ void k_adam(float *w, float *m, float *v, const float *grad, int t, float lr, MlpDev *inf)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float b1 = 0.9f, b2 = 0.999f, e = 1e-8f;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g, vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(b1, (float)t)), vh = vv / (1.f - powf(b2, (float)t));
    const float nw = w[p] - lr * mh / (sqrtf(vh) + e);
    w[p] = nw;
    // BF16 inference copy in the MlpDev layout
    const int nW1 = kMlpH * kMlpIn, nb1 = nW1 + kMlpH, nW2 = nb1 + kMlpH * kMlpH, nb2 = nW2 + kMlpH,
              nW3 = nb2 + kMlpH;
    const uint16_t bb = bf16_bits(nw);
    if (p < nW1) inf->W1[(p / kMlpIn) * 16 + p % kMlpIn] = bb;
    else if (p < nb1) inf->b1[p - nW1] = bf16_float(bb);
    else if (p < nW2) inf->W2[p - nb1] = bb;
    else if (p < nb2) inf->b2[p - nW2] = bf16_float(bb);
    else if (p < nW3) inf->W3[p - nb2] = bf16_float(bb);
    else inf->b3 = bf16_float(bb);
}

int err(swe_ctx *c, int code, const std::string &m)
{
    if (c) c->err = m;
    return code;
}

}  // namespace

constexpr int kTrainBlocks = 512;  // gradient partials: at most this many blocks
constexpr int kMaxDevices = 64;    // devices whose static workspace address is kept

// Per-block gradient partials of swe_trainer_loss_grad_static: a device array
// of fixed size (3.2 MB), one copy per GPU, held until the process ends.  In
// host code this name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device (static_scratch_ptr).
static __device__ __align__(256) float scratch[kTrainBlocks * (kMlpParams + 1)];

struct swe_trainer {
    int dev = 0;
    hipStream_t stream = nullptr;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *partial = nullptr;
    MlpDev *inf = nullptr;
    int t = 0, nblocks = kTrainBlocks;
    std::string err;
};

namespace swe {

int launch_limiter_phi(swe_ctx *c, const void *U, float *out)
{
    if (!c->has_mlp) return err(c, SWE_ERR_STATE, "learned limiter weights not set");
    const int n = c->n_total, B = 256, G = (n + B - 1) / B;
    if (c->tsize == 8) {
        PhiArgs<double> a{n, (const int4 *)c->nbr, (const double4 *)c->he_co, (const double4 *)U,
                          (const MlpDev *)c->mlp, out, c->cfg.g, c->cfg.eps};
        hipLaunchKernelGGL(k_limiter_phi<double>, dim3(G), dim3(B), 0, c->stream, a);
    } else {
        PhiArgs<float> a{n, (const int4 *)c->nbr, (const float4 *)c->he_co, (const float4 *)U,
                         (const MlpDev *)c->mlp, out, (float)c->cfg.g, (float)c->cfg.eps};
        hipLaunchKernelGGL(k_limiter_phi<float>, dim3(G), dim3(B), 0, c->stream, a);
    }
    return hipGetLastError() == hipSuccess ? SWE_OK : err(c, SWE_ERR_DEVICE, "limiter launch failed");
}

}  // namespace swe

extern "C" {

int swe_limiter_set_weights(swe_ctx *c, const float *params)
{
    if (!c || !params) return err(c, SWE_ERR_ARG, "null argument");
    MlpDev w;
    pack_mlp(params, w);
    if (hipSetDevice(c->dev) != hipSuccess) return err(c, SWE_ERR_DEVICE, "hipSetDevice");
    if (hipStreamSynchronize(c->stream) != hipSuccess) return err(c, SWE_ERR_DEVICE, "sync");
    if (!c->mlp && dalloc(c, &c->mlp, sizeof(MlpDev)) != hipSuccess) return err(c, SWE_ERR_OOM, "alloc");
    if (hipMemcpy(c->mlp, &w, sizeof(MlpDev), hipMemcpyHostToDevice) != hipSuccess)
        return err(c, SWE_ERR_DEVICE, "copy");
    c->has_mlp = true;
    c->phi_stale = true;  // the next step evaluates phi with these weights
    return SWE_OK;
}

int swe_limiter_phi(swe_ctx *c, float *dev_phi)
{
    if (!c || !dev_phi) return err(c, SWE_ERR_ARG, "null argument");
    if (!c->has_state) return err(c, SWE_ERR_STATE, "no state");
    if (hipSetDevice(c->dev) != hipSuccess) return err(c, SWE_ERR_DEVICE, "hipSetDevice");
    // straight into the caller's buffer: the phi that the steps between two
    // evaluations reuse stays as it is
    int rc = launch_limiter_phi(c, c->U[c->step_count & 1], dev_phi);
    if (rc != SWE_OK) return rc;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return err(c, SWE_ERR_DEVICE, "sync");
    return SWE_OK;
}

int swe_limiter_pairs(swe_ctx *coarse, swe_ctx *fine, const int32_t *dev_children, float *dev_rec)
{
    if (!coarse || !fine || !dev_children || !dev_rec) return err(coarse, SWE_ERR_ARG, "null argument");
    if (!coarse->has_mesh || !fine->has_state) return err(coarse, SWE_ERR_STATE, "missing mesh or state");
    if (coarse->dev != fine->dev || coarse->tsize != fine->tsize)
        return err(coarse, SWE_ERR_ARG, "contexts differ in device or precision");
    if (hipSetDevice(coarse->dev) != hipSuccess) return err(coarse, SWE_ERR_DEVICE, "hipSetDevice");
    if (hipStreamSynchronize(fine->stream) != hipSuccess) return err(coarse, SWE_ERR_DEVICE, "sync");
    const int n = coarse->n_total, B = 256, G = (n + B - 1) / B;
    void *Uc = coarse->U[0];
    const void *Uf = fine->U[fine->step_count & 1];
    if (hipMemsetAsync(coarse->flag, 0, sizeof(int), coarse->stream) != hipSuccess)
        return err(coarse, SWE_ERR_DEVICE, "memset");
    // the coarse context's state becomes the restriction (with its own bed)
    if (coarse->tsize == 8) {
        hipLaunchKernelGGL(k_restrict<double>, dim3(G), dim3(B), 0, coarse->stream, n, dev_children,
                           fine->n_total, (const double4 *)Uf, (const double *)coarse->bed,
                           (double4 *)Uc, coarse->flag);
        PairArgs<double> a{n, (const int4 *)coarse->nbr, (const double4 *)coarse->he_geo,
                           (const double4 *)coarse->he_dist, (const double4 *)coarse->he_co,
                           (const double4 *)Uc, (const double4 *)Uf,
                           dev_children, fine->n_total, dev_rec, coarse->cfg.g, coarse->cfg.eps};
        hipLaunchKernelGGL(k_pairs<double>, dim3(G), dim3(B), 0, coarse->stream, a);
    } else {
        hipLaunchKernelGGL(k_restrict<float>, dim3(G), dim3(B), 0, coarse->stream, n, dev_children,
                           fine->n_total, (const float4 *)Uf, (const float *)coarse->bed,
                           (float4 *)Uc, coarse->flag);
        PairArgs<float> a{n, (const int4 *)coarse->nbr, (const float4 *)coarse->he_geo,
                          (const float4 *)coarse->he_dist, (const float4 *)coarse->he_co,
                          (const float4 *)Uc, (const float4 *)Uf,
                          dev_children, fine->n_total, dev_rec, (float)coarse->cfg.g,
                          (float)coarse->cfg.eps};
        hipLaunchKernelGGL(k_pairs<float>, dim3(G), dim3(B), 0, coarse->stream, a);
    }
    int bad = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad, coarse->flag, sizeof(int), hipMemcpyDeviceToHost, coarse->stream) != hipSuccess ||
        hipStreamSynchronize(coarse->stream) != hipSuccess)
        return err(coarse, SWE_ERR_DEVICE, "pairs launch failed");
    coarse->step_count = 0;
    if (bad) { coarse->has_state = false; return err(coarse, SWE_ERR_ARG, "child index out of range"); }
    return init_clock(coarse, 0.0);  // the restricted state starts a new run at t = 0
}

int swe_trainer_create(int device, const float *init, swe_trainer **out)
{
    if (!init || !out) return SWE_ERR_ARG;
    *out = nullptr;
    auto *T = new swe_trainer;
    T->dev = device;
    const size_t P = kMlpParams;
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&T->stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&T->w, 4 * P) != hipSuccess || hipMalloc(&T->m, 4 * P) != hipSuccess ||
        hipMalloc(&T->v, 4 * P) != hipSuccess || hipMalloc(&T->grad, 4 * (P + 1)) != hipSuccess ||
        hipMalloc(&T->partial, 4 * (P + 1) * (size_t)T->nblocks) != hipSuccess ||
        hipMalloc(&T->inf, sizeof(MlpDev)) != hipSuccess) {
        swe_trainer_destroy(T);
        return SWE_ERR_DEVICE;
    }
    MlpDev w;
    pack_mlp(init, w);
    std::vector<float> z(P, 0.f);
    if (hipMemcpy(T->w, init, 4 * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(T->m, z.data(), 4 * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(T->v, z.data(), 4 * P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(T->inf, &w, sizeof(MlpDev), hipMemcpyHostToDevice) != hipSuccess) {
        swe_trainer_destroy(T);
        return SWE_ERR_DEVICE;
    }
    *out = T;
    return SWE_OK;
}

void swe_trainer_destroy(swe_trainer *T)
{
    if (!T) return;
    (void)hipSetDevice(T->dev);
    if (T->stream) (void)hipStreamSynchronize(T->stream);
    for (float *p : {T->w, T->m, T->v, T->grad, T->partial})
        if (p) (void)hipFree(p);
    if (T->inf) (void)hipFree(T->inf);
    if (T->stream) (void)hipStreamDestroy(T->stream);
    delete T;
}

// loss and gradient of n records into grad_loss[kMlpParams + 1]: per-block
// partials in `partial` ([nblocks][kMlpParams + 1], every row written before
// it is read, so nothing needs clearing), then a fixed-order reduction
static int launch_grad(const float *params, const float *rec, int32_t n_rec, const int32_t *idx,
                       int32_t n, const float *wv, float *partial, int nblocks, float *grad_loss,
                       hipStream_t stream)
{
    TrainArgs a;
    a.rec = rec; a.idx = idx; a.n = n; a.n_rec = n_rec; a.params = params; a.partial = partial;
    for (int k = 0; k < 4; ++k) a.wv[k] = wv[k];
    const int nchunks = (n + kChunk - 1) / kChunk;
    const int G = nchunks < nblocks ? nchunks : nblocks;
    hipLaunchKernelGGL(k_train_partial, dim3(G), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_train_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, stream,
                       partial, G, n, grad_loss);
    return hipGetLastError() == hipSuccess ? SWE_OK : SWE_ERR_DEVICE;
}

static int trainer_grad(swe_trainer *T, const float *rec, int32_t n_rec, const int32_t *idx,
                        int32_t n, const float *wv)
{
    return launch_grad(T->w, rec, n_rec, idx, n, wv, T->partial, T->nblocks, T->grad, T->stream);
}

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy at its own address).
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[kMaxDevices];

static int static_scratch_ptr(int dev, float **out)
{
    if (dev < 0 || dev >= kMaxDevices) return SWE_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SWE_ERR_DEVICE;
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return SWE_OK;
}

int swe_trainer_loss_grad(swe_trainer *T, const float *rec, int32_t n_rec, const int32_t *idx,
                          int32_t n, const float *wv, float *loss, float *grad_host)
{
    if (!T || !rec || !idx || n <= 0 || n_rec <= 0 || !wv || !loss) return SWE_ERR_ARG;
    if (hipSetDevice(T->dev) != hipSuccess) return SWE_ERR_DEVICE;
    int rc = trainer_grad(T, rec, n_rec, idx, n, wv);
    if (rc != SWE_OK) return rc;
    std::vector<float> g(kMlpParams + 1);
    if (hipMemcpyAsync(g.data(), T->grad, 4 * (kMlpParams + 1), hipMemcpyDeviceToHost, T->stream) != hipSuccess ||
        hipStreamSynchronize(T->stream) != hipSuccess)
        return SWE_ERR_DEVICE;
    *loss = g[kMlpParams];
    if (grad_host) std::memcpy(grad_host, g.data(), 4 * kMlpParams);
    return SWE_OK;
}

int swe_trainer_step(swe_trainer *T, const float *rec, int32_t n_rec, const int32_t *idx,
                     int32_t n, const float *wv, float lr, float *loss)
{
    if (!T || !rec || !idx || n <= 0 || n_rec <= 0 || !wv || !(lr > 0)) return SWE_ERR_ARG;
    if (hipSetDevice(T->dev) != hipSuccess) return SWE_ERR_DEVICE;
    int rc = trainer_grad(T, rec, n_rec, idx, n, wv);
    if (rc != SWE_OK) return rc;
    T->t += 1;
    hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, T->stream, T->w, T->m,
                       T->v, T->grad, T->t, lr, T->inf);
    if (hipGetLastError() != hipSuccess) return SWE_ERR_DEVICE;
    if (loss) {
        if (hipMemcpyAsync(loss, T->grad + kMlpParams, 4, hipMemcpyDeviceToHost, T->stream) != hipSuccess ||
            hipStreamSynchronize(T->stream) != hipSuccess)
            return SWE_ERR_DEVICE;
    }
    return SWE_OK;
}

int swe_trainer_loss_grad_static(const float *dev_params, const float *dev_rec, int32_t n_rec,
                                 const int32_t *dev_idx, int32_t n, const float *wv,
                                 float *dev_grad_loss, void *stream)
{
    if (!dev_params || !dev_rec || !dev_idx || !dev_grad_loss || !wv || n <= 0 || n_rec <= 0)
        return SWE_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SWE_ERR_DEVICE;
    float *partial = nullptr;
    int rc = static_scratch_ptr(dev, &partial);
    if (rc != SWE_OK) return rc;
    return launch_grad(dev_params, dev_rec, n_rec, dev_idx, n, wv, partial, kTrainBlocks,
                       dev_grad_loss, (hipStream_t)stream);
}

int swe_trainer_get_params(swe_trainer *T, float *host_params)
{
    if (!T || !host_params) return SWE_ERR_ARG;
    if (hipSetDevice(T->dev) != hipSuccess || hipStreamSynchronize(T->stream) != hipSuccess ||
        hipMemcpy(host_params, T->w, 4 * kMlpParams, hipMemcpyDeviceToHost) != hipSuccess)
        return SWE_ERR_DEVICE;
    return SWE_OK;
}

}  // extern "C"
