// Internal declarations of the learned-force network kernels (hslb_cnn.hip).
// Nothing here is part of the C ABI.
//
// The network: three 5x5x5 convolutions with bias, 1 -> 32 -> 32 -> 3 channels,
// GELU after the first two.  Input: the packing-fraction field pi sigma^3 n / 6.
// Output: the dimensionless force F_hat; C1 ~= F_hat * v_T^2 (6/pi)^2 4 pi / sigma^4.
//
// Tensors (N = nx*ny*nz nodes, node = x + nx*(y + ny*z), no padding):
//   x      bf16 [N]                     network input
//   a1, a2 bf16 [N][32]  channel-last   activations (convolution inputs)
//   z1, z2 fp32 [N][32]  channel-last   pre-activations (training only)
//   *T     bf16 [32][N]  channel-major  copies for the weight gradients
//   out    fp32 [3][N]                  F_hat
//   d3     bf16 [N][4] / [3][N]         output gradient (4th channel 0)
// x and y are periodic; z is periodic without walls, else zero beyond the array.
// The kernels need nx % 32 == 0 and ny % 4 == 0.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hslb {
namespace cnn {

constexpr int NT = 125;  // taps, t = (dz+2)*25 + (dy+2)*5 + (dx+2)
constexpr int CH = 32;
constexpr int CO = 3;
// canonical FP32 weight vector: W1[32][1][125] b1[32] W2[32][32][125] b2[32] W3[3][32][125] b3[3]
constexpr int OW1 = 0, OB1 = OW1 + CH * NT, OW2 = OB1 + CH, OB2 = OW2 + CH * CH * NT, OW3 = OB2 + CH,
              OB3 = OW3 + CO * CH * NT, NW = OB3 + CO;
static_assert(NW == 144067, "weight count");

struct Geo {
    int nx, ny, nz, zper, N;
};

// Packed MFMA weight operands (bf16 bits), [ksteps][halves][64 lanes][8]:
// forward layers 1-3 and the input-gradient convolutions of layers 2 and 3
// (the B operand everywhere but layer 3's forward, PK_F3: there the A operand
// with rows (output channel, dx), 13 (dy, dz) pair steps per channel half).
// PK_F2, PK_F3 and PK_D2 end in PACK_PAD zero K-steps, so that their kernels'
// prefetch runs past the last step without a branch.
enum PackKind { PK_F1 = 0, PK_F2, PK_F3, PK_D2, PK_D3, PK_COUNT };
constexpr int PACK_PAD = 4;
constexpr int pack_elems(int kind)
{
    return kind == PK_F1 ? 4 * 2 * 512
         : kind == PK_F2 ? (2 * ((NT + 1) / 2) + PACK_PAD) * 2 * 512
         : kind == PK_F3 ? (2 * 13 + PACK_PAD) * 512
         : kind == PK_D2 ? (2 * ((NT + 1) / 2) + PACK_PAD) * 2 * 512
                         : 16 * 2 * 512;
}

// Convolution input layouts: scalar field, 4-channel (3 used), 32-channel.
enum Epi { EPI_GELU = 0, EPI_OUT = 1, EPI_DGELU = 2 };

struct FwdArgs {
    Geo g;
    const uint16_t *in;    // CIN 1: [N]; 4: [N][4]; 32: [N][32]
    const uint16_t *wp;    // packed B operands
    const float *bias;     // [cout] (EPI_GELU, EPI_OUT)
    const float *zsave;    // EPI_DGELU: pre-activation [N][32]
    uint16_t *out_cl;      // bf16 [N][32] (nullable)
    uint16_t *out_cm;      // bf16 [32][N] (nullable)
    float *out_f32;        // EPI_GELU: z [N][32]; EPI_OUT: [3][N]; EPI_DGELU: raw sum [N][32] (nullable)
    int out_zero;          // EPI_OUT: output channels (bit c) written as 0 instead of conv + bias
};

// cin in {1, 4, 32}; cout 32 (two output halves) or 3; epi as above.
hipError_t launch_conv_fwd(hipStream_t s, int cin, int cout, int epi, const FwdArgs &a);

// Weight gradients.  Layer 1: dW1[co][0][t] = sum_n x[n + off_t] g[co][n];
// layers 2/3: dW[co][ci][t] = sum_n actT[ci][n + off_t] gT[co][n], co < cout.
// `partial` is scratch of wgrad_partial_floats(...) floats; the sums are
// written (not accumulated) into dW in canonical order.
size_t wgrad_partial_floats(const Geo &g, int layer);
hipError_t launch_wgrad(hipStream_t s, int layer, const Geo &g, const uint16_t *src, const uint16_t *gT,
                        float *partial, float *dW);
// db[c] = sum_n g[c][n] over channel-major bf16 gradients; `partial` holds
// colsum_partial_floats(...) floats.
size_t colsum_partial_floats(const Geo &g, int nch);
hipError_t launch_colsum(hipStream_t s, const Geo &g, int nch, const uint16_t *gT, float *partial, float *db);

// Packing of the canonical FP32 weights into the MFMA operand layouts.
hipError_t launch_pack(hipStream_t s, int kind, const float *w, uint16_t *out);

// x = bf16(eta_pref * n) from a padded moment field (hz ghost layers).
template <typename TM>
hipError_t launch_eta_input(hipStream_t s, const Geo &g, int hz, double eta_pref, const TM *n, uint16_t *x);
// x = bf16(v) from FP64 host-staged values.
hipError_t launch_to_bf16(hipStream_t s, const double *v, size_t count, uint16_t *out);

// Loss over fluid nodes (wall_lo <= z < nz - wall_hi) of (out - target)^2,
// and the bf16 output gradient 2 (out - target) / (3 n_fluid) in both layouts;
// sq_partial holds one FP64 per block (loss_blocks(g)).
unsigned loss_blocks(const Geo &g);
hipError_t launch_loss(hipStream_t s, const Geo &g, int wall_lo, int wall_hi, const float *out,
                       const float *target, uint16_t *d_cl, uint16_t *d_cm, double *sq_partial);

// Adam on the canonical FP32 weights (step t >= 1).
hipError_t launch_adam(hipStream_t s, int n, float *w, float *m, float *v, const float *g, int t, float lr);

// Residual of the force the surrogate path applies against the exact one
// over fluid nodes: partial sums [blocks][2] of |C1 - pred|^2 and |C1|^2 with
// pred = fs*F_hat + (use_prev ? delta : 0); then delta = C1 - fs*F_hat (0 off
// the fluid).  fhat may be null (0).
unsigned judge_blocks(const Geo &g);
hipError_t launch_judge(hipStream_t s, const Geo &g, int wall_lo, int wall_hi, double fs, const float *fhat,
                        const double *c1, int use_prev, float *delta, double *partial);

// Layout conversions for host-staged test data (FP32 values, channel-major
// [c][N] on the host side): to bf16 channel-last [N][cp] (channels c..cp-1
// zero) and/or bf16 channel-major; back from bf16 or FP32 channel-last.
hipError_t launch_cm_to_bf16(hipStream_t s, const float *in, int c, int cp, int N, uint16_t *out_cl,
                             uint16_t *out_cm);
hipError_t launch_cl_bf16_to_cm(hipStream_t s, const uint16_t *in, int c, int N, float *out);
hipError_t launch_cl_f32_to_cm(hipStream_t s, const float *in, int c, int N, float *out);

// out = s * in, converting between FP32 and FP64.
hipError_t launch_scale_f32_to_f64(hipStream_t st, const float *in, double s, size_t count, double *out);
hipError_t launch_scale_f64_to_f32(hipStream_t st, const double *in, double s, size_t count, float *out);

}  // namespace cnn
}  // namespace hslb
