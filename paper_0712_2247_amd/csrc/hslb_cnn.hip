// Learned-force network on gfx950: 5x5x5 convolutions as implicit GEMMs on
// the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// MFMA operand layout (16x16x32): lane l holds A[m = l%16][k = 8(l/16) .. +8),
// B[k = 8(l/16) .. +8][n = l%16], and accumulates D[m = 4(l/16) + j][n = l%16],
// j = 0..3.  The 8 K-values of a lane are contiguous in K.
//
//  - Forward and input-gradient convolutions: M = 16 consecutive x-nodes of a
//    row, N = output channels, K = (tap, input channel).  The 8 K-values of a
//    lane are 8 channels of one node, a 16-byte load from channel-last bf16
//    activations.  A wave computes 4 rows (z) x 16 nodes against both 16-column
//    output halves; B comes pre-packed in lane order.  The forward layers with
//    32 input channels stage them in two halves of 16 (k_conv_fwd_split), which
//    halves the LDS per block and doubles the resident waves.
//  - Weight gradients: K = nodes, so a lane's 8 K-values are 8 consecutive
//    x-nodes of one channel (channel-major copies).  The x-shift of a tap is
//    taken from aligned 16-byte chunks with 16-bit funnel shifts, wrapping at
//    row ends (nx % 8 == 0 makes the chunks row-aligned).  Per-wave partial
//    sums go to scratch and a second kernel reduces them in a fixed order.
#include "hslb_cnn.hpp"
#include "hslb_internal.hpp"

#include <cmath>

namespace hslb {
namespace cnn {
namespace {

typedef __bf16 bf16x8 __attribute__((__vector_size__(16)));
typedef float f32x4 __attribute__((__vector_size__(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// FP32 -> bf16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint32_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

// FP64 -> bf16 directly: keep 8 significant bits of m in d = m 2^e, ties to even.
__device__ __forceinline__ uint32_t d2bf(double d)
{
    int e;
    const double m = frexp(d, &e);
    const double r = rint(m * 256.0) * (1.0 / 256.0);
    return __float_as_uint((float)ldexp(r, e)) >> 16;
}

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// The standard normal distribution function Phi(z) in FP32, with the Gaussian
// g = exp(-z^2/2) it is built from.  For t = |z|,
//   Phi(-t) = g E(t) / 2,  E(t) = exp(t^2/2) erfc(t / sqrt 2),
// and E = u P(u) with u = 1/(1 + 0.3 t) and P the degree-9 polynomial of
// gen_phi_poly.py (relative error of the fit 3.5e-9 on [0, 16]);
// Phi(z) = 1 - Phi(-z) for z > 0.  z^2 is split exactly (FMA), so that g keeps
// its relative accuracy far in the tail, and the Gaussian is the hardware
// base-2 exponential of c z^2 with the product's rounding carried to first
// order: the result is good to about 6e-7 relative also for z << 0 (where
// 1 + erf(z / sqrt 2) would cancel), with well under half the instructions of
// erfcf.  For z < -13 the Gaussian leaves the normal range (the caller takes
// the reference form there).
__device__ __forceinline__ float phi_cdf_fast(float z, float &g)
{
    const float t = fabsf(z);
    const float q = z * z;
    // g = 2^(c z^2), c = -log2(e) / 2 = CH + CL, z^2 = q + ql: x = q CH rounded, the
    // rest xl = c z^2 - x goes in to first order, g = 2^x (1 + ln2 xl)
    constexpr float CH = -0.7213475108146667f, CL = -9.629815167500055e-09f;
    const float ql = fmaf(z, z, -q);
    const float x = q * CH;
    const float xl = fmaf(q, CH, -x) + fmaf(q, CL, ql * CH);
    g = __builtin_amdgcn_exp2f(x) * fmaf(xl, 0.69314718055994531f, 1.0f);
    const float u = __builtin_amdgcn_rcpf(fmaf(0.3f, t, 1.0f));
    float p = -0.04126075655221939f;
    p = fmaf(p, u, 0.22495317459106445f);
    p = fmaf(p, u, -0.4566359519958496f);
    p = fmaf(p, u, 0.3838684558868408f);
    p = fmaf(p, u, -0.15911298990249634f);
    p = fmaf(p, u, 0.19246527552604675f);
    p = fmaf(p, u, 0.1567239612340927f);
    p = fmaf(p, u, 0.22048330307006836f);
    p = fmaf(p, u, 0.2391420602798462f);
    p = fmaf(p, u, 0.23937346041202545f);
    const float tail = 0.5f * g * (u * p);  // Phi(-t)
    return z < 0.f ? tail : 1.0f - tail;
}

// The reference evaluation, Phi(z) = erfc(-z / sqrt 2) / 2 (a few ulp).
__device__ __forceinline__ float phi_cdf_ref(float z) { return 0.5f * erfcf(-z * 0.70710678118654752f); }

// The forward activations are stored as bf16.  The fast form decides the
// rounding wherever it lies more than 32 FP32 ulps (at least 1.9e-6 relative,
// three times its distance from the reference form) from a bf16 rounding tie;
// the few values nearer a tie (about 1 in 1000) are evaluated again with
// erfcf.  The stored bits are therefore those of the reference form
// z * phi_cdf_ref(z), for a small share of its cost.
__device__ __forceinline__ bool near_bf16_tie(float v)
{
    const uint32_t lo = __float_as_uint(v) & 0xFFFFu;
    return lo - 0x7FE0u < 0x40u;  // lo within 0x8000 - 32 .. 0x8000 + 31
}

// GELU in the reference form, out of line: it runs for about one value in a
// thousand and would otherwise double the epilogue's code.
__device__ __attribute__((noinline)) float gelu_ref(float z) { return z * phi_cdf_ref(z); }

// bf16(GELU(z)), GELU(z) = z Phi(z)
__device__ __forceinline__ uint32_t gelu_bf16(float z)
{
    float g;
    float v = z * phi_cdf_fast(z, g);
    if (near_bf16_tie(v) || z < -13.0f) v = gelu_ref(z);
    return f2bf(v);
}

// bf16(d GELU'(z)), GELU'(z) = Phi(z) + z phi(z), in the reference form: the
// two terms cancel near z = -0.75, where the fast form's error would grow
// past the tie window (the input gradient is a training kernel).
__device__ __forceinline__ uint32_t dgelu_bf16(float d, float z)
{
    return f2bf(d * (phi_cdf_ref(z) + z * expf(-0.5f * z * z) * 0.39894228040143268f));
}

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// z of a tap read: -1 when it falls beyond a walled array.
__device__ __forceinline__ int zsrc(const Geo &g, int z)
{
    if (g.zper) return wrapi(z, g.nz);
    return (z < 0 || z >= g.nz) ? -1 : z;
}

// ------------------------------------------------------------- forward

// A block of 4 waves computes a 16 (x) x 4 (y) x 4 (z) tile of output nodes:
// wave w takes y0 + w, its 4 rows the layers z0 .. z0 + 3.  The input nodes
// the tile reads, 20 x 8 x 8 with the halo of 2, are staged in LDS once (x
// and y wrapped, z wrapped or zero beyond walls); every tap's A operand then
// comes from LDS.  32 input channels are staged as two halves of 32 B per node
// (40 KB each, k_conv_fwd_split); cin = 4: 8 B per node; cin = 1: 2 B.
#ifndef HSLB_CNN_TZ
#define HSLB_CNN_TZ 4
#endif
constexpr int TX = 16, TY = 4, TZ = HSLB_CNN_TZ;
constexpr int KQ = (NT + 1) / 2;  // two-tap K-steps per channel half (k_conv_fwd_split)
constexpr int HX = TX + 4, HY = TY + 4, HZ = TZ + 4, HNODES = HX * HY * HZ;
constexpr int ROWS = TZ;

// v mod n in [0, n) for v within a few periods of the range (halo indices of
// small lattices): adds and subtracts instead of two integer divisions.
__device__ __forceinline__ int mod_pos(int v, int n)
{
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

__host__ __device__ __forceinline__ constexpr int lnode(int hx, int hy, int hz) { return (hz * HY + hy) * HX + hx; }

// LDS byte offsets of the tap pairs of the split-channel convolution relative
// to the output node (16-byte parts): v[2q] is the offset of tap 2q, v[2q + 1]
// that of tap 2q + 1 minus it.  A block reads them as scalar loads; the pad
// tap t = NT reads the node itself (its weights are 0).
struct TapOffsets {
    uint32_t v[2 * KQ];
};
constexpr uint32_t tap_lds_offset(int t) { return t < NT ? (uint32_t)lnode(t % 5, (t / 5) % 5, t / 25) * 16u : 0u; }
constexpr TapOffsets make_tap_offsets()
{
    TapOffsets o{};
    for (int q = 0; q < KQ; ++q) {
        o.v[2 * q] = tap_lds_offset(2 * q);
        o.v[2 * q + 1] = tap_lds_offset(2 * q + 1) - tap_lds_offset(2 * q);
    }
    return o;
}
__constant__ TapOffsets c_tap_offsets = make_tap_offsets();

// Stages channel half hc (16 channels, two 16-byte parts per node, stored
// planar by part) of the block's input halo.  Wave w copies the halo rows
// (hz, hy) = w, w + 4, ...: their source y and z are uniform, and lanes
// 0 .. 2 HX - 1 take the row's HX nodes x 2 parts.
__device__ __forceinline__ void stage_half(const Geo &g, const uint16_t *__restrict__ in, uint16_t *tile, int x0,
                                           int y0, int z0, int hc, int lane)
{
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int hx = lane >> 1, pt = lane & 1;
    const bool act = lane < 2 * HX;
    const size_t col = (size_t)(act ? wrapi(x0 - 2 + hx, g.nx) : 0) * 32 + 16 * hc + 8 * pt;
    for (int row = w; row < HY * HZ; row += 4) {
        const int hy = row % HY, hz = row / HY;
        const int zr = z0 - 2 + hz;
        const int zs = g.zper ? mod_pos(zr, g.nz) : ((zr < 0 || zr >= g.nz) ? -1 : zr);
        const size_t rbase = (size_t)g.nx * (mod_pos(y0 - 2 + hy, g.ny) + (size_t)g.ny * (zs < 0 ? 0 : zs)) * 32;
        if (act) {
            u32x4 v = {0u, 0u, 0u, 0u};
            if (zs >= 0) v = *(const u32x4 *)(in + rbase + col);
            ((u32x4 *)tile)[pt * HNODES + row * HX + hx] = v;
        }
    }
}


template <int CIN>
__device__ __forceinline__ void stage_tile(const Geo &g, const uint16_t *__restrict__ in, uint16_t *tile, int x0,
                                           int y0, int z0)
{
    static_assert(CIN == 1 || CIN == 4, "32-channel inputs are staged by halves (stage_half)");
    for (int node = threadIdx.x; node < HNODES; node += 256) {
        const int hx = node % HX, hy = (node / HX) % HY, hz = node / (HX * HY);
        const int zr = z0 - 2 + hz;
        const int zs = g.zper ? mod_pos(zr, g.nz) : ((zr < 0 || zr >= g.nz) ? -1 : zr);
        size_t src = 0;
        if (zs >= 0) src = (size_t)wrapi(x0 - 2 + hx, g.nx) + (size_t)g.nx * (mod_pos(y0 - 2 + hy, g.ny) + (size_t)g.ny * zs);
        if constexpr (CIN == 4) {
            u32x2 v = {0u, 0u};
            if (zs >= 0) v = *(const u32x2 *)(in + src * 4);
            ((u32x2 *)tile)[node] = v;
        } else {
            tile[node] = zs >= 0 ? in[src] : (uint16_t)0;
        }
    }
}

// Tap offsets of the A operands of k_conv_fwd, in tile nodes relative to the
// lane's node, per K-step s and lane group lg: CIN 1, taps 32 s + 8 lg + e
// (e = 0..7); CIN 4, taps 8 s + 2 lg + q (q = 0, 1).  Taps past the last read
// the node itself against zero weights.  A lane reads its step's offsets with
// one or two 16-byte loads instead of dividing each tap index by 5 and 25.
struct FwdTapOffsets {
    uint32_t c1[4][4][8];
    uint32_t c4[16][4][4];  // q = 0, 1 used; padded to 16 bytes
};
constexpr uint32_t tap_node(int t) { return t < NT ? (uint32_t)lnode(t % 5, (t / 5) % 5, t / 25) : 0u; }
constexpr FwdTapOffsets make_fwd_tap_offsets()
{
    FwdTapOffsets o{};
    for (int s = 0; s < 4; ++s)
        for (int lg = 0; lg < 4; ++lg)
            for (int e = 0; e < 8; ++e) o.c1[s][lg][e] = tap_node(32 * s + 8 * lg + e);
    for (int s = 0; s < 16; ++s)
        for (int lg = 0; lg < 4; ++lg)
            for (int q = 0; q < 2; ++q) o.c4[s][lg][q] = tap_node(8 * s + 2 * lg + q);
    return o;
}
__constant__ FwdTapOffsets c_fwd_taps = make_fwd_tap_offsets();

// A operand of K-step s for the lane's node `node` (tile index of row r) from
// the step's tap offsets.
template <int CIN>
__device__ __forceinline__ u32x4 lds_a(const uint16_t *tile, int node, const uint32_t (&off)[8])
{
    u32x4 v = {0u, 0u, 0u, 0u};
    if constexpr (CIN == 4) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const u32x2 w2 = ((const u32x2 *)tile)[node + off[q]];
            v[2 * q] = w2[0];
            v[2 * q + 1] = w2[1];
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e >> 1] |= (uint32_t)tile[node + off[e]] << (16 * (e & 1));
    }
    return v;
}

// GELU epilogue of a forward layer with 32 output channels: lane (li, lg)
// holds acc[r][h][j] of node (x0 + 4 lg + j, y0 + w, z0 + r), channel 16 h + li.
// The activations go through LDS, so that the channel-last copy leaves as
// whole 16-byte node parts and the channel-major copy as runs of consecutive
// nodes, instead of one scattered 2-byte store per value.  `ot` holds
// TX * TY * TZ * 32 bf16 (16 KB) of LDS that no wave reads any more; tile-local
// node l = (r TY + y) TX + x.
__device__ __forceinline__ void gelu_epilogue(const FwdArgs &a, const Geo &g, uint16_t *ot, const f32x4 (&acc)[ROWS][2],
                                              int x0, int y0, int z0, int rows, int w, int li, int lg)
{
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int rowbase = g.nx * ((y0 + w) + g.ny * (z0 + r));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = 16 * h + li;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float zz = acc[r][h][j] + a.bias[c];
                ot[((r * TY + w) * TX + 4 * lg + j) * 32 + c] = (uint16_t)gelu_bf16(zz);
                if (a.out_f32 && r < rows) a.out_f32[(size_t)(rowbase + x0 + 4 * lg + j) * 32 + c] = zz;
            }
        }
    }
    __syncthreads();
    constexpr int TN = TX * TY * TZ;
    if (a.out_cl) {
        for (int q = threadIdx.x; q < TN * 4; q += 256) {
            const int l = q >> 2, pt = q & 3;
            const int x = l % TX, y = (l / TX) % TY, r = l / (TX * TY);
            if (r < rows) {
                const size_t node = (size_t)(x0 + x) + (size_t)g.nx * ((y0 + y) + (size_t)g.ny * (z0 + r));
                *(u32x4 *)(a.out_cl + node * 32 + 8 * pt) = *(const u32x4 *)(ot + l * 32 + 8 * pt);
            }
        }
    }
    if (a.out_cm) {
        for (int q = threadIdx.x; q < TN * 32; q += 256) {
            const int c = q / TN, l = q - c * TN;
            const int x = l % TX, y = (l / TX) % TY, r = l / (TX * TY);
            if (r < rows) {
                const size_t node = (size_t)(x0 + x) + (size_t)g.nx * ((y0 + y) + (size_t)g.ny * (z0 + r));
                a.out_cm[(size_t)c * g.N + node] = ot[l * 32 + c];
            }
        }
    }
}

// Layer 1 forward (1 -> 32 channels, GELU epilogue) and the input gradient of
// layer 3 (its 3 output-gradient channels padded to 4 -> 32, GELU' epilogue):
// the block's whole input halo fits LDS (2 or 8 bytes per node).  The B
// operands (the same for every block, so cache hits) are loaded PD K-steps
// ahead into a register ring; rows past the end of a partial z tile are
// computed on the staged zeros or wrapped layers and not stored, which keeps
// the loop free of branches.
template <int CIN, int EPI>
__global__ __launch_bounds__(256) void k_conv_fwd(FwdArgs a)
{
    static_assert((CIN == 1 && EPI == EPI_GELU) || (CIN == 4 && EPI == EPI_DGELU),
                  "layer 1 forward, layer 3 input gradient");
    constexpr int NH = 2;
    constexpr int KS = CIN == 4 ? 16 : 4;
    __shared__ __attribute__((aligned(16))) uint16_t tile[HNODES * CIN];
    const Geo g = a.g;
    const int nxb = g.nx / TX, nyb = g.ny / TY;
    const int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int zb = b / (nxb * nyb);
    const int rem = b - zb * nxb * nyb;
    const int yb = rem / nxb;
    const int x0 = (rem - yb * nxb) * TX, y0 = yb * TY, z0 = zb * TZ;
    stage_tile<CIN>(g, a.in, tile, x0, y0, z0);
    __syncthreads();

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int rows = min(ROWS, g.nz - z0);  // the last z tile may be partial
    f32x4 acc[ROWS][NH];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int h = 0; h < NH; ++h) acc[r][h] = (f32x4){0.f, 0.f, 0.f, 0.f};

    constexpr int PD = 8;
    auto load_b = [&](int s, int h) { return *(const u32x4 *)(a.wp + ((size_t)(s * NH + h) * 64 + lane) * 8); };
    u32x4 bq[PD][NH];
#pragma unroll
    for (int q = 0; q < PD; ++q)
#pragma unroll
        for (int h = 0; h < NH; ++h) bq[q][h] = q < KS ? load_b(q, h) : (u32x4){0u, 0u, 0u, 0u};
    for (int s0 = 0; s0 < KS; s0 += PD) {
#pragma unroll
        for (int q = 0; q < PD; ++q) {
            const int s = s0 + q;
            if (s < KS) {
                uint32_t off[8];
                if constexpr (CIN == 1) {
                    const u32x4 o0 = *(const u32x4 *)&c_fwd_taps.c1[s][lg][0];
                    const u32x4 o1 = *(const u32x4 *)&c_fwd_taps.c1[s][lg][4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        off[e] = o0[e];
                        off[4 + e] = o1[e];
                    }
                } else {
                    const u32x4 o0 = *(const u32x4 *)&c_fwd_taps.c4[s][lg][0];
#pragma unroll
                    for (int e = 0; e < 4; ++e) off[e] = o0[e];
                    off[4] = off[5] = off[6] = off[7] = 0u;
                }
                bf16x8 av[ROWS], bw[NH];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) av[r] = as_bf(lds_a<CIN>(tile, lnode(li, w, r), off));
#pragma unroll
                for (int h = 0; h < NH; ++h) {
                    bw[h] = as_bf(bq[q][h]);
                    if (s + PD < KS) bq[q][h] = load_b(s + PD, h);
                }
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
#pragma unroll
                    for (int h = 0; h < NH; ++h)
                        acc[r][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[r], bw[h], acc[r][h], 0, 0, 0);
            }
        }
    }

    if constexpr (EPI == EPI_GELU) {
        __shared__ __attribute__((aligned(16))) uint16_t ot[TX * TY * TZ * 32];
        gelu_epilogue(a, g, ot, acc, x0, y0, z0, rows, w, li, lg);
    } else {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            if (r >= rows) continue;
            const int rowbase = g.nx * ((y0 + w) + g.ny * (z0 + r));
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int c = 16 * h + li;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int node = rowbase + x0 + 4 * lg + j;
                    const float v = acc[r][h][j];
                    const uint32_t bits = dgelu_bf16(v, a.zsave[(size_t)node * 32 + c]);
                    if (a.out_f32) a.out_f32[(size_t)node * 32 + c] = v;
                    if (a.out_cl) a.out_cl[(size_t)node * 32 + c] = (uint16_t)bits;
                    if (a.out_cm) a.out_cm[(size_t)c * g.N + node] = (uint16_t)bits;
                }
            }
        }
    }
}

// Forward layer 2 (32 -> 32 channels, GELU) and its input gradient
// (transposed weights, GELU' epilogue), with the input channels in two halves
// of 16.  The staged halo then holds 32 B per node (40 KB instead of
// 80 KB), so four blocks share a compute unit, twice the resident waves of the
// 64-byte halo, which hides the latencies of the LDS and weight reads.  A K-step
// of 32 covers two taps x 16 channels: lane group lg takes tap 2q + lg/2 and
// channels 8 (lg % 2) .. + 8 of the half; the weights come packed in that order
// (PK_F2, PK_D2).  Output layout and epilogues as k_conv_fwd.  The K-loop
// carries no branch and no per-lane index arithmetic: the tap offsets come
// from a constant table through scalar loads, the B ring runs on over the
// zero-padded end of the pack, and a ring slot is refilled after its products
// are issued (no register copies, no wait on a load just issued).  On the
// 64x64x136 slit layer 2 takes 141 us (40 % of the BF16 peak; 188 us with
// per-lane tap division and guarded loads, 249 us with the 64-byte halo).
template <int NH, int EPI>
__global__ __launch_bounds__(256, 4) void k_conv_fwd_split(FwdArgs a)
{
    static_assert(NH == 2 && (EPI == EPI_GELU || EPI == EPI_DGELU), "layer 2 forward and input gradient");
    __shared__ __attribute__((aligned(16))) uint16_t tile[HNODES * 16];
    const Geo g = a.g;
    const int nxb = g.nx / TX, nyb = g.ny / TY;
    const int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int zb = b / (nxb * nyb);
    const int rem = b - zb * nxb * nyb;
    const int yb = rem / nxb;
    const int x0 = (rem - yb * nxb) * TX, y0 = yb * TY, z0 = zb * TZ;

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int part = lg & 1, second = lg >> 1;
    const int rows = min(ROWS, g.nz - z0);
    f32x4 acc[ROWS][NH];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int h = 0; h < NH; ++h) acc[r][h] = (f32x4){0.f, 0.f, 0.f, 0.f};

    // B operands: a ring of PD K-steps loaded ahead, over the steps of both
    // channel halves in a row (the packs end in PACK_PAD zero steps).
    constexpr int PD = 3;
    static_assert(KQ % PD == 0 && PD <= PACK_PAD, "the prefetch ring runs on across the halves");
    auto load_b = [&](int sq, int h) { return *(const u32x4 *)(a.wp + ((size_t)(sq * NH + h) * 64 + lane) * 8); };
    u32x4 bq[PD][NH];
#pragma unroll
    for (int q = 0; q < PD; ++q)
#pragma unroll
        for (int h = 0; h < NH; ++h) bq[q][h] = load_b(q, h);
    // A operands: the LDS byte offset of a lane's node (x0 + li, y0 + w, z0)
    // of its 16-byte part, plus the offset of its tap of the pair.
    const uint32_t lane_base = (uint32_t)(part * HNODES + lnode(li, w, 0)) * 16u;
    const uint32_t second_mask = second ? ~0u : 0u;
    constexpr uint32_t ROW_BYTES = HX * HY * 16;
    for (int hc = 0; hc < 2; ++hc) {
        if (hc) __syncthreads();  // every wave is done with the first half
        stage_half(g, a.in, tile, x0, y0, z0, hc, lane);
        __syncthreads();
#pragma unroll 1
        for (int q0 = 0; q0 < KQ; q0 += PD) {
#pragma unroll
            for (int qq = 0; qq < PD; ++qq) {
                const int q = q0 + qq;
                const uint32_t t0 = __builtin_amdgcn_readfirstlane(c_tap_offsets.v[2 * q]);
                const uint32_t dt = __builtin_amdgcn_readfirstlane(c_tap_offsets.v[2 * q + 1]);
                const uint32_t off = lane_base + t0 + (dt & second_mask);
                bf16x8 av[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
                    av[r] = as_bf(*(const u32x4 *)((const char *)tile + off + r * ROW_BYTES));
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
#pragma unroll
                    for (int h = 0; h < NH; ++h)
                        acc[r][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[r], as_bf(bq[qq][h]), acc[r][h], 0, 0, 0);
                // refill the ring slot once its products are issued, so that
                // the load lands in the same registers
#pragma unroll
                for (int h = 0; h < NH; ++h) bq[qq][h] = load_b(hc * KQ + q + PD, h);
            }
        }
    }

    if constexpr (EPI == EPI_GELU) {
        static_assert(TX * TY * TZ * 32 <= HNODES * 16, "the block's activations fit the halo buffer");
        gelu_epilogue(a, g, tile, acc, x0, y0, z0, rows, w, li, lg);
    } else {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            if (r >= rows) continue;
            const int rowbase = g.nx * ((y0 + w) + g.ny * (z0 + r));
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int c = 16 * h + li;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int node = rowbase + x0 + 4 * lg + j;
                    const float v = acc[r][h][j];
                    const uint32_t bits = dgelu_bf16(v, a.zsave[(size_t)node * 32 + c]);
                    if (a.out_f32) a.out_f32[(size_t)node * 32 + c] = v;
                    if (a.out_cl) a.out_cl[(size_t)node * 32 + c] = (uint16_t)bits;
                    if (a.out_cm) a.out_cm[(size_t)c * g.N + node] = (uint16_t)bits;
                }
            }
        }
    }
}

// Layer 3 forward (32 -> 3 channels) with (output channel, dx) on the M
// dimension of the products instead of the 16 x-nodes: M = 15 used of 16
// rows (c, dx), N = 16 input columns x', K = 16 channels x two (dy, dz) taps.
// The partial sums P[(c, dx)][x'] of a row then give
//   out[c][x] = b[c] + sum_dx P[(c, dx)][x + dx]
// through LDS.  A wave covers the 20 input columns of its 16 output nodes with
// two N-tiles (32 columns, 20 used) and 4 z-rows, so a K-step is 8 products
// against 1 weight fragment, where the node-major form (3 of 16 output
// columns used) needs 2.4 times the products and LDS reads.  Halo staging and
// the block's tile as in k_conv_fwd_split.  Weights packed as PK_F3.  On the
// 64x64x136 slit: 61 us, against 91 us for the node-major form in the
// split-channel kernel (69 us with the K loop rolled).
constexpr int KD = 13;  // (dy, dz) pair steps per channel half: 25 taps + 1 pad

struct DyDzOffsets {
    uint32_t v[2 * KD];
};
constexpr DyDzOffsets make_dydz_offsets()
{
    DyDzOffsets o{};
    for (int q = 0; q < KD; ++q)
        for (int p = 0; p < 2; ++p) {
            const int i = 2 * q + p;
            o.v[i] = i < 25 ? (uint32_t)lnode(0, i % 5, i / 5) * 16u : 0u;
        }
    return o;
}
__constant__ DyDzOffsets c_dydz_offsets = make_dydz_offsets();

__global__ __launch_bounds__(256, 4) void k_conv_out(FwdArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t tile[HNODES * 16];
    const Geo g = a.g;
    const int nxb = g.nx / TX, nyb = g.ny / TY;
    const int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int zb = b / (nxb * nyb);
    const int rem = b - zb * nxb * nyb;
    const int yb = rem / nxb;
    const int x0 = (rem - yb * nxb) * TX, y0 = yb * TY, z0 = zb * TZ;

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int part = lg & 1, second = lg >> 1;
    const int rows = min(ROWS, g.nz - z0);
    f32x4 acc[ROWS][2];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[r][nt] = (f32x4){0.f, 0.f, 0.f, 0.f};

    // B operand: column x' = li + 16 nt of the halo (x0 - 2 + x'); the columns
    // past the halo's 20 are not needed and read its last one.
    uint32_t col_base[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
        col_base[nt] = (uint32_t)(part * HNODES + lnode(min(li + 16 * nt, HX - 1), w, 0)) * 16u;
    const uint32_t second_mask = second ? ~0u : 0u;
    constexpr uint32_t ROW_BYTES = HX * HY * 16;
    auto load_a = [&](int sq) { return *(const u32x4 *)(a.wp + ((size_t)sq * 64 + lane) * 8); };
    u32x4 wq = load_a(0);
    for (int hc = 0; hc < 2; ++hc) {
        if (hc) __syncthreads();
        stage_half(g, a.in, tile, x0, y0, z0, hc, lane);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < KD; ++q) {  // unrolled: the next step's LDS reads start early
            const uint32_t t0 = __builtin_amdgcn_readfirstlane(c_dydz_offsets.v[2 * q]);
            const uint32_t t1 = __builtin_amdgcn_readfirstlane(c_dydz_offsets.v[2 * q + 1]);
            const uint32_t off = t0 + ((t1 - t0) & second_mask);
            const bf16x8 wa = as_bf(wq);
            wq = load_a(hc * KD + q + 1);  // the pack ends in PACK_PAD zero steps
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    const bf16x8 bv = as_bf(*(const u32x4 *)((const char *)tile + col_base[nt] + off + r * ROW_BYTES));
                    acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, bv, acc[r][nt], 0, 0, 0);
                }
        }
    }

    // P[r][m][x'] of the wave through LDS (the halo is no longer read), then
    // out[c][x0 + i] = b[c] + sum_dx P[r][5 c + dx][i + dx].
    __syncthreads();
    float *P = (float *)tile + w * (ROWS * 16 * 32);
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) P[(r * 16 + 4 * lg + j) * 32 + li + 16 * nt] = acc[r][nt][j];
    __syncthreads();
    for (int k = lane; k < ROWS * CO * 16; k += 64) {
        const int i = k & 15, c = (k >> 4) % CO, r = k / (16 * CO);
        if (r >= rows) continue;
        float v = a.bias[c];
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) v += P[(r * 16 + 5 * c + dx) * 32 + i + dx];
        const size_t node = (size_t)(x0 + i) + (size_t)g.nx * ((y0 + w) + (size_t)g.ny * (z0 + r));
        a.out_f32[(size_t)c * g.N + node] = (a.out_zero >> c) & 1 ? 0.f : v;
    }
}

// ---------------------------------------------------- weight gradients

// 8 consecutive elements starting at element `sh` (in -2..2) of the chunk
// `cur`, continuing into `prv` / `nxt`.
__device__ __forceinline__ u32x4 shifted(const u32x4 &prv, const u32x4 &cur, const u32x4 &nxt, int sh)
{
    u32x4 o;
    if (sh == 0) return cur;
    if (sh == 2) {
        o[0] = cur[1];
        o[1] = cur[2];
        o[2] = cur[3];
        o[3] = nxt[0];
    } else if (sh == -2) {
        o[0] = prv[3];
        o[1] = cur[0];
        o[2] = cur[1];
        o[3] = cur[2];
    } else if (sh == 1) {
        o[0] = (cur[0] >> 16) | (cur[1] << 16);
        o[1] = (cur[1] >> 16) | (cur[2] << 16);
        o[2] = (cur[2] >> 16) | (cur[3] << 16);
        o[3] = (cur[3] >> 16) | (nxt[0] << 16);
    } else {
        o[0] = (prv[3] >> 16) | (cur[0] << 16);
        o[1] = (cur[0] >> 16) | (cur[1] << 16);
        o[2] = (cur[1] >> 16) | (cur[2] << 16);
        o[3] = (cur[2] >> 16) | (cur[3] << 16);
    }
    return o;
}

// rows (y, z) of the lattice split into chunks of rpw rows
struct RowSplit {
    int rows, rpw, chunks;
};

__host__ __device__ inline RowSplit row_split(const Geo &g, int max_chunks)
{
    RowSplit r;
    r.rows = g.ny * g.nz;
    const int c = r.rows < max_chunks ? r.rows : max_chunks;
    r.rpw = (r.rows + c - 1) / c;
    r.chunks = (r.rows + r.rpw - 1) / r.rpw;
    return r;
}

constexpr int WG_CHUNKS_CH = 64;    // layers 2, 3: waves = 25 tap rows x chunks
constexpr int WG_CHUNKS_TAP = 1024; // layer 1: waves = chunks

// Layers 2 and 3: M = input channel (2 x 16), N = output channel (NB x 16),
// K = nodes.  Wave = (tap row (dz, dy), chunk of lattice rows); the 5 dx taps
// share the three chunks loaded per channel.
// partial[wave][5][32][16 NB]
template <int NB>
__global__ __launch_bounds__(256) void k_wgrad_ch(Geo g, RowSplit rs, int cout, const uint16_t *__restrict__ actT,
                                                  const uint16_t *__restrict__ gT, float *__restrict__ partial)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wave >= 25 * rs.chunks) return;
    const int gq = wave % 25, chunk = wave / 25;
    const int dz = gq / 5 - 2, dy = gq % 5 - 2;
    const int li = lane & 15, lg = lane >> 4;
    f32x4 acc[5][2][NB];
#pragma unroll
    for (int d = 0; d < 5; ++d)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[d][mi][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};

    const int r0 = chunk * rs.rpw, r1 = min(rs.rows, r0 + rs.rpw);
    for (int row = r0; row < r1; ++row) {
        const int y = row % g.ny, z = row / g.ny;
        const int zs = zsrc(g, z + dz);
        if (zs < 0) continue;  // the tap reads beyond the walls: zero
        const size_t srow = (size_t)g.nx * (wrapi(y + dy, g.ny) + g.ny * zs);
        const size_t orow = (size_t)g.nx * (y + g.ny * z);
        for (int x0 = 0; x0 < g.nx; x0 += 32) {
            const int xc = x0 + 8 * lg;
            bf16x8 bv[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int co = 16 * nb + li;
                u32x4 w = {0u, 0u, 0u, 0u};
                if (co < cout) w = *(const u32x4 *)(gT + (size_t)co * g.N + orow + xc);
                bv[nb] = as_bf(w);
            }
            const int xp = xc == 0 ? g.nx - 8 : xc - 8, xn = xc + 8 == g.nx ? 0 : xc + 8;
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) {
                const uint16_t *base = actT + (size_t)(16 * mi + li) * g.N + srow;
                const u32x4 prv = *(const u32x4 *)(base + xp);
                const u32x4 cur = *(const u32x4 *)(base + xc);
                const u32x4 nxt = *(const u32x4 *)(base + xn);
#pragma unroll
                for (int d = 0; d < 5; ++d) {
                    const bf16x8 av = as_bf(shifted(prv, cur, nxt, d - 2));
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[d][mi][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nb], acc[d][mi][nb], 0, 0, 0);
                }
            }
        }
    }
    float *out = partial + (size_t)wave * 5 * 32 * 16 * NB;
#pragma unroll
    for (int d = 0; d < 5; ++d)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ci = 16 * mi + 4 * lg + j, co = 16 * nb + li;
                    out[((size_t)d * 32 + ci) * 16 * NB + co] = acc[d][mi][nb][j];
                }
}

// dW[co][ci][t] = sum over chunks, t = gq * 5 + d; threads run over co
// fastest, then ci, so that neighbouring threads read neighbouring partials
__global__ __launch_bounds__(256) void k_wgrad_ch_reduce(int chunks, int nb16, int cout, const float *__restrict__ partial,
                                                         float *__restrict__ dW)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= cout * 32 * NT) return;
    const int co = i % cout, ci = (i / cout) % 32, t = i / (cout * 32);
    const int gq = t / 5, d = t % 5;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c)
        s += partial[(((size_t)(c * 25 + gq) * 5 + d) * 32 + ci) * nb16 + co];
    dW[(co * 32 + ci) * NT + t] = (float)s;
}

// Layer 1: M = tap (8 x 16, taps >= 125 zero), N = output channel (2 x 16),
// K = nodes.  Each lane's tap has its own shift.  partial[wave][128][32]
__global__ __launch_bounds__(256) void k_wgrad_tap(Geo g, RowSplit rs, const uint16_t *__restrict__ x,
                                                   const uint16_t *__restrict__ gT, float *__restrict__ partial)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wave >= rs.chunks) return;
    const int li = lane & 15, lg = lane >> 4;
    f32x4 acc[8][2];
#pragma unroll
    for (int mi = 0; mi < 8; ++mi)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mi][nb] = (f32x4){0.f, 0.f, 0.f, 0.f};

    const int r0 = wave * rs.rpw, r1 = min(rs.rows, r0 + rs.rpw);
    for (int row = r0; row < r1; ++row) {
        const int y = row % g.ny, z = row / g.ny;
        const size_t orow = (size_t)g.nx * (y + g.ny * z);
        for (int x0 = 0; x0 < g.nx; x0 += 32) {
            const int xc = x0 + 8 * lg;
            bf16x8 bv[2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) bv[nb] = as_bf(*(const u32x4 *)(gT + (size_t)(16 * nb + li) * g.N + orow + xc));
            const int xp = xc == 0 ? g.nx - 8 : xc - 8, xn = xc + 8 == g.nx ? 0 : xc + 8;
#pragma unroll
            for (int mi = 0; mi < 8; ++mi) {
                const int t = 16 * mi + li;
                u32x4 v = {0u, 0u, 0u, 0u};
                if (t < NT) {
                    const int dz = t / 25 - 2, dy = (t / 5) % 5 - 2, dx = t % 5 - 2;
                    const int zs = zsrc(g, z + dz);
                    if (zs >= 0) {
                        const uint16_t *base = x + (size_t)g.nx * (wrapi(y + dy, g.ny) + g.ny * zs);
                        const u32x4 cur = *(const u32x4 *)(base + xc);
                        const u32x4 prv = dx < 0 ? *(const u32x4 *)(base + xp) : cur;
                        const u32x4 nxt = dx > 0 ? *(const u32x4 *)(base + xn) : cur;
                        v = shifted(prv, cur, nxt, dx);
                    }
                }
                const bf16x8 av = as_bf(v);
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                    acc[mi][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nb], acc[mi][nb], 0, 0, 0);
            }
        }
    }
    float *out = partial + (size_t)wave * 128 * 32;
#pragma unroll
    for (int mi = 0; mi < 8; ++mi)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int j = 0; j < 4; ++j) out[(16 * mi + 4 * lg + j) * 32 + 16 * nb + li] = acc[mi][nb][j];
}

// dW1[co][0][t]; threads run over co fastest (neighbouring partials)
__global__ __launch_bounds__(256) void k_wgrad_tap_reduce(int chunks, const float *__restrict__ partial,
                                                          float *__restrict__ dW)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 32 * NT) return;
    const int co = i % 32, t = i / 32;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += partial[((size_t)c * 128 + t) * 32 + co];
    dW[co * NT + t] = (float)s;
}

// --------------------------------------------------------- reductions

__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

constexpr int COLSUM_CHUNKS = 64;

// partial[c][chunk]
__global__ __launch_bounds__(256) void k_colsum(Geo g, const uint16_t *__restrict__ gT, float *__restrict__ partial)
{
    __shared__ double red[4];
    const int c = blockIdx.y, chunk = blockIdx.x;
    const int per = (g.N + COLSUM_CHUNKS - 1) / COLSUM_CHUNKS;
    const int n0 = chunk * per, n1 = min(g.N, n0 + per);
    double s = 0.0;
    for (int n = n0 + (int)threadIdx.x; n < n1; n += 256) s += (double)bf2f(gT[(size_t)c * g.N + n]);
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) partial[c * COLSUM_CHUNKS + chunk] = (float)t;
}

__global__ void k_colsum_reduce(int nch, const float *__restrict__ partial, float *__restrict__ db)
{
    const int c = threadIdx.x;
    if (c >= nch) return;
    double s = 0.0;
    for (int k = 0; k < COLSUM_CHUNKS; ++k) s += (double)partial[c * COLSUM_CHUNKS + k];
    db[c] = (float)s;
}

// ------------------------------------------------------------ packing

__global__ __launch_bounds__(256) void k_pack(int kind, const float *__restrict__ w, uint16_t *__restrict__ out, int total)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int e = idx & 7, lane = (idx >> 3) & 63, rest = idx >> 9;
    const int li = lane & 15, lg = lane >> 4;
    const int H = kind == PK_F3 ? 1 : 2;
    const int h = rest % H, s = rest / H;
    const int col = 16 * h + li;
    float v = 0.f;
    if (kind == PK_F1) {
        const int t = 32 * s + 8 * lg + e;
        if (t < NT) v = w[OW1 + col * NT + t];
    } else if (kind == PK_F2) {
        // channel half hc, two-tap step q: lane group lg holds tap 2q + lg/2,
        // channels 16 hc + 8 (lg % 2) .. + 8 (k_conv_fwd_split); zero padding
        // steps after the second half
        const int hc = s / KQ, q = s - hc * KQ, t = 2 * q + (lg >> 1);
        if (hc < 2 && t < NT) v = w[OW2 + (col * CH + 16 * hc + 8 * (lg & 1) + e) * NT + t];
    } else if (kind == PK_F3) {
        // A operand of k_conv_out: row li = (output channel li / 5, dx li % 5),
        // channel half hc, (dy, dz) pair step q: lane group lg holds tap
        // (dy, dz) number 2q + lg/2 (dz major), channels 16 hc + 8 (lg % 2) .. + 8
        const int hc = s / KD, q = s - hc * KD, i = 2 * q + (lg >> 1);
        const int c = li / 5, dx = li % 5;
        if (hc < 2 && c < CO && i < 25) v = w[OW3 + (c * CH + 16 * hc + 8 * (lg & 1) + e) * NT + (i / 5) * 25 + (i % 5) * 5 + dx];
    } else if (kind == PK_D2) {
        // transposed, tap-flipped layer-2 weights in the split order of PK_F2
        const int hc = s / KQ, q = s - hc * KQ, t = 2 * q + (lg >> 1);
        if (hc < 2 && t < NT) v = w[OW2 + ((16 * hc + 8 * (lg & 1) + e) * CH + col) * NT + (NT - 1 - t)];
    } else {
        const int t = 8 * s + 2 * lg + (e >> 2), cf = e & 3;
        if (t < NT && cf < CO) v = w[OW3 + (cf * CH + col) * NT + (NT - 1 - t)];
    }
    out[idx] = (uint16_t)f2bf(v);
}

// --------------------------------------------------------------- misc

template <typename TM>
__global__ __launch_bounds__(256) void k_eta_input(Geo g, int hz, double eta_pref, const TM *__restrict__ n,
                                                   uint16_t *__restrict__ x)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= g.N) return;
    const int plane = g.nx * g.ny;
    x[i] = (uint16_t)d2bf(eta_pref * (double)n[i + hz * plane]);
}

__global__ __launch_bounds__(256) void k_to_bf16(const double *__restrict__ v, size_t count, uint16_t *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) out[i] = (uint16_t)d2bf(v[i]);
}

__global__ __launch_bounds__(256) void k_loss(Geo g, int wall_lo, int wall_hi, float scale, const float *__restrict__ out,
                                              const float *__restrict__ target, uint16_t *__restrict__ d_cl,
                                              uint16_t *__restrict__ d_cm, double *__restrict__ sq_partial)
{
    __shared__ double red[4];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double sq = 0.0;
    if (i < g.N) {
        const int z = i / (g.nx * g.ny);
        const bool fl = z >= wall_lo && z < g.nz - wall_hi;
#pragma unroll
        for (int c = 0; c < CO; ++c) {
            const float d = fl ? out[(size_t)c * g.N + i] - target[(size_t)c * g.N + i] : 0.f;
            sq += (double)d * (double)d;
            const uint16_t b = (uint16_t)f2bf(d * scale);
            d_cl[(size_t)i * 4 + c] = b;
            d_cm[(size_t)c * g.N + i] = b;
        }
        d_cl[(size_t)i * 4 + 3] = 0;
    }
    const double t = block_sum(sq, red);
    if (threadIdx.x == 0) sq_partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_adam(int n, float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ g, float c1, float c2, float lr)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// Residual of the force the surrogate path applies, fs F_hat + delta_old
// (delta_old only with use_prev), against the exact C1 over fluid nodes; then
// delta = C1 - fs F_hat (in place: each node reads its old value first).
__global__ __launch_bounds__(256) void k_judge(Geo g, int wall_lo, int wall_hi, double fs, const float *__restrict__ fhat,
                                               const double *__restrict__ c1, int use_prev, float *__restrict__ delta,
                                               double *__restrict__ partial)
{
    __shared__ double red[4];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (i < g.N) {
        const int z = i / (g.nx * g.ny);
        const bool fl = z >= wall_lo && z < g.nz - wall_hi;
#pragma unroll
        for (int c = 0; c < CO; ++c) {
            const size_t k = (size_t)c * g.N + i;
            const double e = c1[k];
            const double f = fhat ? fs * (double)fhat[k] : 0.0;
            if (fl) {
                const double pred = f + (use_prev ? (double)delta[k] : 0.0);
                a += (e - pred) * (e - pred);
                b += e * e;
            }
            delta[k] = fl ? (float)(e - f) : 0.f;
        }
    }
    const double ta = block_sum(a, red);
    const double tb = block_sum(b, red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = ta;
        partial[2 * blockIdx.x + 1] = tb;
    }
}

__global__ __launch_bounds__(256) void k_f32_to_f64(const float *__restrict__ in, double s, size_t count,
                                                    double *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) out[i] = s * (double)in[i];
}

__global__ __launch_bounds__(256) void k_f64_to_f32(const double *__restrict__ in, double s, size_t count,
                                                    float *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) out[i] = (float)(s * in[i]);
}

__global__ __launch_bounds__(256) void k_cm_to_bf16(const float *__restrict__ in, int c, int cp, int N,
                                                    uint16_t *__restrict__ out_cl, uint16_t *__restrict__ out_cm)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)cp * N) return;
    const int n = (int)(i / cp), k = (int)(i % cp);
    const uint16_t b = k < c ? (uint16_t)f2bf(in[(size_t)k * N + n]) : (uint16_t)0;
    if (out_cl) out_cl[i] = b;
    if (out_cm && k < c) out_cm[(size_t)k * N + n] = b;
}

__global__ __launch_bounds__(256) void k_cl_bf16_to_cm(const uint16_t *__restrict__ in, int c, int N, float *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)c * N) return;
    const int k = (int)(i / N), n = (int)(i % N);
    out[i] = bf2f(in[(size_t)n * c + k]);
}

__global__ __launch_bounds__(256) void k_cl_f32_to_cm(const float *__restrict__ in, int c, int N, float *__restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)c * N) return;
    const int k = (int)(i / N), n = (int)(i % N);
    out[i] = in[(size_t)n * c + k];
}

inline unsigned nblocks(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_conv_fwd(hipStream_t s, int cin, int cout, int epi, const FwdArgs &a)
{
    const int blocks = (a.g.nx / TX) * (a.g.ny / TY) * ((a.g.nz + TZ - 1) / TZ);
    const dim3 grid(blocks), blk(256);
    const int nh = cout == 32 ? 2 : 1;
    if (cin == 1 && nh == 2 && epi == EPI_GELU) {
        hipLaunchKernelGGL((k_conv_fwd<1, EPI_GELU>), grid, blk, 0, s, a);
        return hipGetLastError();
    }
    if (cin == 32 && nh == 2 && epi == EPI_GELU) {
        hipLaunchKernelGGL((k_conv_fwd_split<2, EPI_GELU>), grid, blk, 0, s, a);
        return hipGetLastError();
    }
    if (cin == 32 && nh == 2 && epi == EPI_DGELU) {
        hipLaunchKernelGGL((k_conv_fwd_split<2, EPI_DGELU>), grid, blk, 0, s, a);
        return hipGetLastError();
    }
    if (cin == 32 && nh == 1 && epi == EPI_OUT) {
        hipLaunchKernelGGL(k_conv_out, grid, blk, 0, s, a);
        return hipGetLastError();
    }
    if (cin == 4 && nh == 2 && epi == EPI_DGELU) {
        hipLaunchKernelGGL((k_conv_fwd<4, EPI_DGELU>), grid, blk, 0, s, a);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

size_t wgrad_partial_floats(const Geo &g, int layer)
{
    if (layer == 1) return (size_t)row_split(g, WG_CHUNKS_TAP).chunks * 128 * 32;
    const int nb = layer == 2 ? 2 : 1;
    return (size_t)25 * row_split(g, WG_CHUNKS_CH).chunks * 5 * 32 * 16 * nb;
}

hipError_t launch_wgrad(hipStream_t s, int layer, const Geo &g, const uint16_t *src, const uint16_t *gT,
                        float *partial, float *dW)
{
    if (layer == 1) {
        const RowSplit rs = row_split(g, WG_CHUNKS_TAP);
        hipLaunchKernelGGL(k_wgrad_tap, dim3((rs.chunks + 3) / 4), dim3(256), 0, s, g, rs, src, gT, partial);
        hipLaunchKernelGGL(k_wgrad_tap_reduce, dim3(nblocks(32 * NT)), dim3(256), 0, s, rs.chunks, partial, dW);
        return hipGetLastError();
    }
    const RowSplit rs = row_split(g, WG_CHUNKS_CH);
    const unsigned grid = (unsigned)((25 * rs.chunks + 3) / 4);
    if (layer == 2) {
        hipLaunchKernelGGL(k_wgrad_ch<2>, dim3(grid), dim3(256), 0, s, g, rs, CH, src, gT, partial);
        hipLaunchKernelGGL(k_wgrad_ch_reduce, dim3(nblocks(CH * 32 * NT)), dim3(256), 0, s, rs.chunks, 32, CH, partial, dW);
    } else {
        hipLaunchKernelGGL(k_wgrad_ch<1>, dim3(grid), dim3(256), 0, s, g, rs, CO, src, gT, partial);
        hipLaunchKernelGGL(k_wgrad_ch_reduce, dim3(nblocks(CO * 32 * NT)), dim3(256), 0, s, rs.chunks, 16, CO, partial, dW);
    }
    return hipGetLastError();
}

size_t colsum_partial_floats(const Geo &, int nch) { return (size_t)nch * COLSUM_CHUNKS; }

hipError_t launch_colsum(hipStream_t s, const Geo &g, int nch, const uint16_t *gT, float *partial, float *db)
{
    hipLaunchKernelGGL(k_colsum, dim3(COLSUM_CHUNKS, nch), dim3(256), 0, s, g, gT, partial);
    hipLaunchKernelGGL(k_colsum_reduce, dim3(1), dim3(64), 0, s, nch, partial, db);
    return hipGetLastError();
}

hipError_t launch_pack(hipStream_t s, int kind, const float *w, uint16_t *out)
{
    const int total = pack_elems(kind);
    hipLaunchKernelGGL(k_pack, dim3(nblocks(total)), dim3(256), 0, s, kind, w, out, total);
    return hipGetLastError();
}

template <typename TM>
hipError_t launch_eta_input(hipStream_t s, const Geo &g, int hz, double eta_pref, const TM *n, uint16_t *x)
{
    hipLaunchKernelGGL(k_eta_input<TM>, dim3(nblocks(g.N)), dim3(256), 0, s, g, hz, eta_pref, n, x);
    return hipGetLastError();
}
template hipError_t launch_eta_input<float>(hipStream_t, const Geo &, int, double, const float *, uint16_t *);
template hipError_t launch_eta_input<double>(hipStream_t, const Geo &, int, double, const double *, uint16_t *);

hipError_t launch_to_bf16(hipStream_t s, const double *v, size_t count, uint16_t *out)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(nblocks(count)), dim3(256), 0, s, v, count, out);
    return hipGetLastError();
}

unsigned loss_blocks(const Geo &g) { return nblocks(g.N); }

hipError_t launch_loss(hipStream_t s, const Geo &g, int wall_lo, int wall_hi, const float *out, const float *target,
                       uint16_t *d_cl, uint16_t *d_cm, double *sq_partial)
{
    const long nf = (long)g.nx * g.ny * (g.nz - wall_lo - wall_hi);
    const float scale = (float)(2.0 / (3.0 * (double)nf));
    hipLaunchKernelGGL(k_loss, dim3(loss_blocks(g)), dim3(256), 0, s, g, wall_lo, wall_hi, scale, out, target, d_cl, d_cm,
                       sq_partial);
    return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, int n, float *w, float *m, float *v, const float *g, int t, float lr)
{
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, t)));
    hipLaunchKernelGGL(k_adam, dim3(nblocks(n)), dim3(256), 0, s, n, w, m, v, g, c1, c2, lr);
    return hipGetLastError();
}

unsigned judge_blocks(const Geo &g) { return nblocks(g.N); }

hipError_t launch_cm_to_bf16(hipStream_t s, const float *in, int c, int cp, int N, uint16_t *out_cl, uint16_t *out_cm)
{
    hipLaunchKernelGGL(k_cm_to_bf16, dim3(nblocks((size_t)cp * N)), dim3(256), 0, s, in, c, cp, N, out_cl, out_cm);
    return hipGetLastError();
}

hipError_t launch_cl_bf16_to_cm(hipStream_t s, const uint16_t *in, int c, int N, float *out)
{
    hipLaunchKernelGGL(k_cl_bf16_to_cm, dim3(nblocks((size_t)c * N)), dim3(256), 0, s, in, c, N, out);
    return hipGetLastError();
}

hipError_t launch_cl_f32_to_cm(hipStream_t s, const float *in, int c, int N, float *out)
{
    hipLaunchKernelGGL(k_cl_f32_to_cm, dim3(nblocks((size_t)c * N)), dim3(256), 0, s, in, c, N, out);
    return hipGetLastError();
}

hipError_t launch_scale_f32_to_f64(hipStream_t st, const float *in, double s, size_t count, double *out)
{
    hipLaunchKernelGGL(k_f32_to_f64, dim3(nblocks(count)), dim3(256), 0, st, in, s, count, out);
    return hipGetLastError();
}

hipError_t launch_scale_f64_to_f32(hipStream_t st, const double *in, double s, size_t count, float *out)
{
    hipLaunchKernelGGL(k_f64_to_f32, dim3(nblocks(count)), dim3(256), 0, st, in, s, count, out);
    return hipGetLastError();
}

hipError_t launch_judge(hipStream_t s, const Geo &g, int wall_lo, int wall_hi, double fs, const float *fhat,
                        const double *c1, int use_prev, float *delta, double *partial)
{
    hipLaunchKernelGGL(k_judge, dim3(judge_blocks(g)), dim3(256), 0, s, g, wall_lo, wall_hi, fs, fhat, c1, use_prev,
                       delta, partial);
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace hslb
