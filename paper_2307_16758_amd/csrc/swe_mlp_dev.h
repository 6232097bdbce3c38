// Inference of the learned slope limiter on the matrix cores (an addition of
// this library; the paper's limiters are the classic ones of Sec. 6.2.3):
// the network 14 -> 32 -> 32 -> 1 (ReLU, ReLU, sigmoid) on BF16 operands
// with FP32 accumulation, shared by the stand-alone limiter kernel and the
// stage kernel that evaluates it inside its first phase.
//
// A wave evaluates 64 half-edges at a time, one per lane: every lane writes
// its half-edge's 16 BF16 inputs (14 features, a zero pad, the eligibility
// flag) to a row of a wave-private LDS block of 64 rows, and the wave runs
// the rows as four MFMA tiles of 16 columns.  All layers are computed
// transposed (units x half-edges): the weights are the A operand, the layer
// input the B operand and the bias the accumulator's initial value, so a
// layer's accumulator (lane: four units of one half-edge) is, after ReLU and
// BF16 rounding, the next layer's B operand as it stands.  The hidden layer
// and the output layer take all 32 inputs in one v_mfma_f32_16x16x32_bf16:
// a lane's eight K slots hold the units of its two accumulators of the layer
// before (units 4q..4q+3 and 16+4q..16+4q+3 for lane group q), and the A
// operand takes its weights in the same order.  The output layer of tile q
// holds W3 in row 4q of its A operand (zeros elsewhere), so its 16 results
// are element 0 of lanes 16q..16q+15: one select per lane then gathers the
// four tiles, and the result of row l is in lane l.  Each tile keeps an
// accumulator of its own, so a non-finite value stays in its tile.  Every
// result depends only on its own column, so a half-edge's output is the
// same bits whichever rows share its tiles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "swe_kernels.h"

namespace swe {

typedef short s2v __attribute__((ext_vector_type(2)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// Inference weights: BF16 matrices (layer-1 K padded 14 -> 16 with zeros),
// biases and the output layer as floats holding BF16-rounded values.
struct MlpDev {
    uint16_t W1[kMlpH * 16];
    uint16_t W2[kMlpH * kMlpH];
    float b1[kMlpH], b2[kMlpH], W3[kMlpH], b3, pad[3];
};

// round-to-nearest-even float -> bfloat16 bits (finite inputs)
__host__ __device__ inline uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_float(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
__device__ __forceinline__ float bf16_round(float f) { return bf16_float(bf16_bits(f)); }
// the same rounding (to nearest, ties to even) by the hardware conversion
__device__ __forceinline__ uint16_t bf16_bits_hw(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_round_hw(float f) { return (float)(__bf16)f; }

// ReLU of an MFMA accumulator (4 values), rounded to BF16 and packed as
// half of the next layer's B operand: two values per conversion, then the
// ReLU on the packed BF16 values as signed 16-bit integers (a negative BF16
// value, -0 included, is a negative integer; the order of non-negative ones
// is their numeric order), the same bits as rounding max(x, 0)
__device__ __forceinline__ s4v relu_bf16x4(f4v d)
{
    const f2v lo = {d[0], d[1]}, hi = {d[2], d[3]};
    const s2v z = {0, 0};
    const s2v a = __builtin_elementwise_max(__builtin_bit_cast(s2v, __builtin_convertvector(lo, bf2v)), z);
    const s2v b = __builtin_elementwise_max(__builtin_bit_cast(s2v, __builtin_convertvector(hi, bf2v)), z);
    const s4v r = {a[0], a[1], b[0], b[1]};
    return r;
}

__device__ __forceinline__ bf8v cat8(s4v a, s4v b)
{
    const s8v v = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    return __builtin_bit_cast(bf8v, v);
}

// The lanes of one wave exchange data through its own LDS rows without a
// block barrier: the wave's LDS operations are processed in order, and this
// keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One lane's share of the weights, in operand order (lane: column col =
// lane & 15 of A, K group kq = 4 (lane >> 4)).
struct MlpLane {
    s4v W1[2];       // layer 1, units nt*16 + col, inputs kq..kq+3
    bf8v W2[2];      // layer 2, units nt*16 + col, inputs kq..kq+3 and 16+kq..16+kq+3
    bf8v W3;         // output weights of the same inputs (row 4q of tile q only)
    f4v b1[2], b2[2];  // biases of units nt*16 + kq..kq+3
    float b3;
};

__device__ __forceinline__ MlpLane mlp_lane(const MlpDev *w, int lane)
{
    const int col = lane & 15, kq = (lane >> 4) * 4;
    MlpLane L;
    s4v w3[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        L.W1[nt] = *(const s4v *)&w->W1[(nt * 16 + col) * 16 + kq];
        L.W2[nt] = cat8(*(const s4v *)&w->W2[(nt * 16 + col) * 32 + kq],
                        *(const s4v *)&w->W2[(nt * 16 + col) * 32 + 16 + kq]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            L.b1[nt][j] = w->b1[nt * 16 + kq + j];
            L.b2[nt][j] = w->b2[nt * 16 + kq + j];
            w3[nt][j] = (short)bf16_bits_hw(w->W3[nt * 16 + kq + j]);
        }
    }
    L.W3 = cat8(w3[0], w3[1]);
    L.b3 = w->b3;
    return L;
}

// Input row of a half-edge: 14 features in BF16, a zero pad and the flag
// (BF16 one when the half-edge is evaluated; its weight column is zero).
__device__ __forceinline__ void mlp_write_row(uint16_t *row, const float f[kMlpIn], bool ok)
{
    unsigned u[8];
#pragma unroll
    for (int i = 0; i < 7; ++i) {  // two values per conversion (round to nearest even)
        const f2v p = {f[2 * i], f[2 * i + 1]};
        u[i] = __builtin_bit_cast(unsigned, __builtin_convertvector(p, bf2v));
    }
    u[7] = ok ? 0x3F800000u : 0u;
    uint4 *r = (uint4 *)row;
    r[0] = make_uint4(u[0], u[1], u[2], u[3]);
    r[1] = make_uint4(u[4], u[5], u[6], u[7]);
}

// Pre-activation of the output unit for row `lane` of the wave's 64 rows X
// (16 BF16 values each; written by the wave and synchronised before).
__device__ __forceinline__ float mlp_rows_z(const MlpLane &L, const uint16_t (*X)[16], int lane)
{
    const int col = lane & 15, kq = (lane >> 4) * 4;
    const bf8v zero8 = {};
    // b3 in element 0 of every lane: rows 0, 4, 8 and 12 of the accumulator
    const f4v c3 = {L.b3, 0.f, 0.f, 0.f};
    const int grp = lane >> 4;
    float z = 0.0f;
    // one tile at a time (not unrolled: four tiles in flight would hold four
    // sets of accumulators)
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        // B: inputs kq..kq+3 of row q * 16 + col
        const s4v xb = *(const s4v *)&X[q * 16 + col][kq];
        const f4v d0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(L.W1[0], xb, L.b1[0], 0, 0, 0);
        const f4v d1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(L.W1[1], xb, L.b1[1], 0, 0, 0);
        const bf8v h = cat8(relu_bf16x4(d0), relu_bf16x4(d1));
        const f4v e0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.W2[0], h, L.b2[0], 0, 0, 0);
        const f4v e1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.W2[1], h, L.b2[1], 0, 0, 0);
        const bf8v gv = cat8(relu_bf16x4(e0), relu_bf16x4(e1));
        const f4v o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(col == 4 * q ? L.W3 : zero8, gv, c3, 0, 0, 0);
        z = grp == q ? o[0] : z;
    }
    return z;
}

// phi of an evaluated half-edge; NaN (not evaluated) where the half-edge is
// not reconstructed to second order, so a stage that does reconstruct it
// falls back to minmod
__device__ __forceinline__ float mlp_phi(float z, bool ok)
{
    return ok ? 1.0f / (1.0f + expf(-z)) : __builtin_nanf("");
}

}  // namespace swe
