// HIP kernels of the hard-sphere lattice Boltzmann step for gfx950.
//
// One step (equation (10) of the paper) runs as five kernels on the stream:
//   k_moments  populations -> n, j                      (equation (8))
//   k_rowsum,  n -> coarse-grained packing fraction      (ball of radius sigma/2,
//   k_ballsum     as row-segment sums: two passes)
//   k_gfield   eta_bar -> contact values g2 on the 7 sub-lattices of pair
//              midpoints (lattice nodes, edge, face centres)
//   k_collide  shell-sum force C^(1) of equation (12) + n g, BGK collision with
//              the second-order equilibrium (11) and first-order source, push
//              streaming with halfway bounce-back
//
// Storage: populations SoA [19][pop_stride] in TF (float or double), kept
// relative to the layer means of each population (a per-layer reference table,
// refreshed now and then) so that FP32 storage keeps the small lateral
// deviations rather than the layered state itself; every sum, the equilibrium subtraction and the shell sum are
// FP64 in registers.  Moment fields (n, j, eta_bar, G) are TM, padded with hz layers
// in z that hold zeros beyond walls or periodic ghost copies.
#include "hslb_internal.hpp"

#include <algorithm>
#include <mutex>
#include <utility>
#include <cmath>
#include <type_traits>

// Tuning switch (compile-time): 1 evaluates the shell sum in FP64 whatever the
// storage precision.  FP32 arithmetic on FP32 fields was measured: within 2 %
// of the time (the kernel is bound by its ~130 vector-memory reads per node,
// not by arithmetic) and up to 15x the profile error in narrow dense slits,
// where the rounding of the large layering terms meets the small viscous ones.
#ifndef HSLB_FORCE_FP64
#define HSLB_FORCE_FP64 1
#endif


namespace hslb {

namespace {


// The collision takes opposite velocities in pairs (i, i + 1), i odd.
constexpr bool odd_pairs_opposite()
{
    for (int i = 1; i < NQ; i += 2)
        if (OPP[i] != i + 1 || CX[i] != -CX[i + 1] || CY[i] != -CY[i + 1] || CZ[i] != -CZ[i + 1]) return false;
    return true;
}
static_assert(odd_pairs_opposite(), "D3Q19 order: every odd velocity is followed by its opposite");

__device__ __forceinline__ constexpr double wq(int i)
{
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// floor(sigma / sqrt(2)): the largest l with 2 l^2 <= sigma^2.
__host__ __device__ constexpr int ell_of(int sigma)
{
    int l = 0;
    while (2 * (l + 1) * (l + 1) <= sigma * sigma) ++l;
    return l;
}

__host__ __device__ constexpr int floordiv2(int d) { return (d - (d & 1)) / 2; }

template <int D>
__device__ __forceinline__ int wrapc(int v, int n)
{
    int w = v + D;
    if constexpr (D > 0) w = (w >= n) ? w - n : w;
    if constexpr (D < 0) w = (w < 0) ? w + n : w;
    return w;
}

__device__ __forceinline__ int wrapr(int w, int n)
{
    w = (w < 0) ? w + n : w;
    return (w >= n) ? w - n : w;
}

__device__ __forceinline__ double g2_of(double eta, int model)
{
    const double om = 1.0 - eta;
    const double num = model ? (1.0 - 0.5 * eta) : (1.0 - 0.5 * eta + 0.25 * eta * eta);
    return num / (om * om * om);
}

// One vector access to the interleaved (n, jx, jy, jz) of a node.
typedef float f32v4 __attribute__((ext_vector_type(4)));
typedef double f64v4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void load4(const float *p, float q[4])
{
    const f32v4 v = *(const f32v4 *)p;
    q[0] = v[0], q[1] = v[1], q[2] = v[2], q[3] = v[3];
}
__device__ __forceinline__ void load4(const double *p, double q[4])
{
    const f64v4 v = *(const f64v4 *)p;
    q[0] = v[0], q[1] = v[1], q[2] = v[2], q[3] = v[3];
}
__device__ __forceinline__ void store4(float *p, float a, float b, float c, float d) { *(f32v4 *)p = (f32v4){a, b, c, d}; }
__device__ __forceinline__ void store4(double *p, double a, double b, double c, double d)
{
    *(f64v4 *)p = (f64v4){a, b, c, d};
}

// Store v at padded z = z + hz and, for a periodic z axis, at every ghost layer
// congruent to it modulo nz.
template <typename TM>
__device__ __forceinline__ void store_padded(const LatticeDev &L, TM *dst, int rem, int z, TM v)
{
    if (!L.zper) {
        dst[rem + L.plane * (z + L.hz)] = v;
        return;
    }
    int p = z + L.hz;
    while (p - L.nz >= 0) p -= L.nz;
    for (; p < L.nz + 2 * L.hz; p += L.nz) dst[rem + L.plane * p] = v;
}

// store_padded with non-temporal stores (fields written once and read by a
// later kernel of a lattice beyond the last-level cache).
template <typename TM>
__device__ __forceinline__ void store_padded_nt(const LatticeDev &L, TM *dst, int rem, int z, TM v)
{
    if (!L.zper) {
        __builtin_nontemporal_store(v, dst + rem + L.plane * (z + L.hz));
        return;
    }
    int p = z + L.hz;
    while (p - L.nz >= 0) p -= L.nz;
    for (; p < L.nz + 2 * L.hz; p += L.nz) __builtin_nontemporal_store(v, dst + rem + L.plane * p);
}

// The interleaved (n, j) of a node into the padded field [..][4], with the
// periodic images in the ghost layers as store_padded.
template <typename TM>
__device__ __forceinline__ void store_padded4(const LatticeDev &L, TM *dst, int rem, int z, TM a, TM b, TM c, TM d)
{
    if (!L.zper) {
        store4(dst + 4 * ((size_t)rem + (size_t)L.plane * (z + L.hz)), a, b, c, d);
        return;
    }
    int p = z + L.hz;
    while (p - L.nz >= 0) p -= L.nz;
    for (; p < L.nz + 2 * L.hz; p += L.nz) store4(dst + 4 * ((size_t)rem + (size_t)L.plane * p), a, b, c, d);
}

// store_padded4 with non-temporal stores.
template <typename TM>
__device__ __forceinline__ void store_padded4_nt(const LatticeDev &L, TM *dst, int rem, int z, TM a, TM b, TM c,
                                                 TM d)
{
    auto st = [&](int p) {
        TM *q = dst + 4 * ((size_t)rem + (size_t)L.plane * p);
        __builtin_nontemporal_store(a, q);
        __builtin_nontemporal_store(b, q + 1);
        __builtin_nontemporal_store(c, q + 2);
        __builtin_nontemporal_store(d, q + 3);
    };
    if (!L.zper) {
        st(z + L.hz);
        return;
    }
    int p = z + L.hz;
    while (p - L.nz >= 0) p -= L.nz;
    for (; p < L.nz + 2 * L.hz; p += L.nz) st(p);
}

__device__ __forceinline__ bool is_fluid_z(const LatticeDev &L, int z)
{
    return L.zper || (z >= L.wall_lo && z < L.nz - L.wall_hi);
}

// Populations are stored relative to a per-layer reference: the value kept
// for direction i at a node of layer z is f_i - ref[z][i], where ref[z] holds
// the layer means of the 19 populations (refreshed now and then).  ref tables
// are [nz][19] doubles.
__device__ __forceinline__ const double *layer_ref(const double *__restrict__ ref, int z) { return ref + 19 * z; }

// --------------------------------------------------------------------- init

// Local equilibrium (11) of (n, u) as full FP64 populations [19][N] (0 on
// solid nodes): the staging form from which initial populations are stored.
__global__ __launch_bounds__(256) void k_feq(LatticeDev L, const double *__restrict__ n,
                                             const double *__restrict__ u, double *__restrict__ out)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    const int z = id / L.plane;
    const bool fl = is_fluid_z(L, z);
    const double nn = fl ? n[id] : 0.0;
    const double ux = fl ? u[id] : 0.0, uy = fl ? u[L.N + id] : 0.0, uz = fl ? u[2 * L.N + id] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        out[(size_t)i * L.N + id] = fl ? wq(i) * nn * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu) : 0.0;
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Layer means of the 19 populations of layer z (0 on solid layers), summed in
// FP64 in a fixed order: from full FP64 populations [19][N] (ref == nullptr)
// or from stored ones plus the current reference.
template <typename TF>
__device__ __forceinline__ void d_layer_means(const LatticeDev &L, const TF *__restrict__ f, int stride,
                                              const double *__restrict__ ref, double *__restrict__ out, int z)
{
    __shared__ double red[4][NQ];
    double s[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) s[i] = 0.0;
    const bool fl = is_fluid_z(L, z);
    if (fl) {
        for (int r = threadIdx.x; r < L.plane; r += 256) {
            const int id = z * L.plane + r;
#pragma unroll
            for (int i = 0; i < NQ; ++i) s[i] += (double)f[(size_t)i * stride + id];
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const double t = wave_sum(s[i]);
        if (lane == 0) red[wv][i] = t;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        const int i = threadIdx.x;
        const double t = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
        const double base = ref ? layer_ref(ref, z)[i] : 0.0;
        out[19 * z + i] = fl ? base + t / (double)L.plane : 0.0;
    }
}

template <typename TF>
__global__ __launch_bounds__(256) void k_layer_means(LatticeDev L, const TF *__restrict__ f, int stride,
                                                     const double *__restrict__ ref, double *__restrict__ out)
{
    d_layer_means(L, f, stride, ref, out, blockIdx.x);
}

// ------------------------------------------------------------------ moments

// Node r of layer z (0 <= r < plane).  Called with a block-uniform z from the
// layer-indexed grid, so the reference row is read through scalar loads.
template <typename TF, typename TM>
__device__ __forceinline__ TM d_moments(const LatticeDev &L, const double *__restrict__ nref,
                                        const TF *__restrict__ f, const Fields<TM> &fld, int z, int r,
                                        bool write_n = true, bool nt = false)
{
    const int id = z * L.plane + r;
    double n = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    if (is_fluid_z(L, z)) {
        const double *rf = layer_ref(nref, z);
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const double fi = (double)f[(size_t)i * L.pop_stride + id] + rf[i];
            n += fi;
            if (CX[i] > 0) jx += fi;
            if (CX[i] < 0) jx -= fi;
            if (CY[i] > 0) jy += fi;
            if (CY[i] < 0) jy -= fi;
            if (CZ[i] > 0) jz += fi;
            if (CZ[i] < 0) jz -= fi;
        }
    }
    if (write_n) store_padded(L, fld.n, r, z, (TM)n);
    if (nt)
        store_padded4_nt(L, fld.nj, r, z, (TM)n, (TM)jx, (TM)jy, (TM)jz);
    else
        store_padded4(L, fld.nj, r, z, (TM)n, (TM)jx, (TM)jy, (TM)jz);
    return (TM)n;
}

// grid (ceil(plane / 256), nz): x = chunk of the layer, y = layer
template <typename TF, typename TM>
__global__ __launch_bounds__(256) void k_moments(LatticeDev L, const double *__restrict__ nref,
                                                 const TF *__restrict__ f, Fields<TM> fld)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < L.plane) d_moments(L, nref, f, fld, (int)blockIdx.y, r);
}

// Moments fused with the row sums of the two-pass ball sum: the block holds
// whole x-rows of layer z (nx divides 256, plane a multiple of 256), so each
// node's row sums rs[w], w = 0..R, come from the block's densities in LDS.
// They are written at the padded layer of z and, for a periodic z axis, at
// its images within the padded range the ball sum reads, [hz - R, nz + hz + R).
template <int SIG, typename TM>
__device__ __forceinline__ void block_rowsums(const LatticeDev &L, const TM *sn, TM *__restrict__ rs, int z, int r,
                                              bool nt = false);

template <int SIG, typename TF, typename TM>
__global__ __launch_bounds__(256) void k_moments_rs(LatticeDev L, const double *__restrict__ nref,
                                                    const TF *__restrict__ f, Fields<TM> fld, TM *__restrict__ rs,
                                                    int write_n, int nt)
{
    __shared__ TM sn[256];
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int z = (int)blockIdx.y;
    sn[threadIdx.x] = d_moments(L, nref, f, fld, z, r, write_n != 0, nt != 0);
    __syncthreads();
    block_rowsums<SIG>(L, sn, rs, z, r, nt != 0);
}

// Row sums rs[w], w = 0..R, of node r of layer z from the block's densities in
// LDS (the block holds whole x-rows of the layer), written at the padded layer
// of z and, for a periodic z axis, at its images within the padded range the
// ball sum reads, [hz - R, nz + hz + R).
template <int SIG, typename TM>
__device__ __forceinline__ void block_rowsums(const LatticeDev &L, const TM *sn, TM *__restrict__ rs, int z, int r,
                                              bool nt)
{
    constexpr int R = SIG / 2;
    const int x = (int)threadIdx.x % L.nx;
    const int row = (int)threadIdx.x - x;
    TM acc[R + 1];
    acc[0] = sn[threadIdx.x];
#pragma unroll
    for (int w = 1; w <= R; ++w) acc[w] = acc[w - 1] + (sn[row + wrapr(x - w, L.nx)] + sn[row + wrapr(x + w, L.nx)]);
    int p0 = z + L.hz, p1 = p0;
    if (L.zper) {
        while (p0 - L.nz >= L.hz - R) p0 -= L.nz;
        p1 = L.nz + L.hz + R - 1;
    }
    for (int p = p0; p <= p1; p += L.nz) {
        const size_t q = (size_t)r + (size_t)L.plane * p;
#pragma unroll
        for (int w = 0; w <= R; ++w) {
            if (nt)
                __builtin_nontemporal_store(acc[w], rs + (size_t)w * L.fld_stride + q);
            else
                rs[(size_t)w * L.fld_stride + q] = acc[w];
        }
    }
}

// ------------------------------------------------- coarse-grained density

// The ball sum in two passes.  Pass 1 (k_rowsum): for every node of the
// padded z range the ball needs, the sums of n over the centred x segments of
// half-width w = 0..R, rs[w] (at most 2R+1 reads per node).  Pass 2
// (k_ballsum): eta_bar as the sum over the (oy, oz) rows of the ball of
// rs[w(oy, oz)], one read per row (49 for sigma = 8 instead of 257).
__host__ __device__ constexpr int isqrt_floor(int v)
{
    int r = 0;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// Row sums of node r (0 <= r < plane) of padded layer zl (0 .. nz + 2R - 1).
template <int SIG, typename TM>
__device__ __forceinline__ void d_rowsum(const LatticeDev &L, const Fields<TM> &fld, TM *__restrict__ rs, int zl, int r)
{
    constexpr int R = SIG / 2;
    const int y = r / L.nx;
    const int x = r - y * L.nx;
    const int p = r + L.plane * (zl - R + L.hz);
    const TM *row = fld.n + (p - x);
    TM acc = row[x];
    rs[p] = acc;
#pragma unroll
    for (int w = 1; w <= R; ++w) {
        acc += row[wrapr(x - w, L.nx)] + row[wrapr(x + w, L.nx)];
        rs[(size_t)w * L.fld_stride + p] = acc;
    }
}

// grid (ceil(plane / 256), nz + 2R)
template <int SIG, typename TM>
__global__ __launch_bounds__(256) void k_rowsum(LatticeDev L, Fields<TM> fld, TM *__restrict__ rs)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < L.plane) d_rowsum<SIG>(L, fld, rs, (int)blockIdx.y, r);
}

// eta_bar of node r (0 <= r < plane) of layer z.
template <int SIG, typename TM>
__device__ __forceinline__ void d_ballsum(const LatticeDev &L, double eta_pref, const Fields<TM> &fld,
                                          const TM *__restrict__ rs, int z, int r)
{
    const int y = r / L.nx;
    const int x = r - y * L.nx;
    constexpr int R = SIG / 2;
    double s = 0.0;
#pragma unroll
    for (int oy = -R; oy <= R; ++oy) {
        const int yy = wrapr(y + oy, L.ny);
        const TM *col = rs + x + L.nx * (yy + L.ny * (z + L.hz));
#pragma unroll
        for (int oz = -R; oz <= R; ++oz) {
            constexpr int S2 = SIG * SIG;
            const int rem2 = S2 - 4 * (oy * oy + oz * oz);
            if (rem2 >= 0) {
                const int w = isqrt_floor(rem2 / 4);
                s += (double)col[(size_t)w * L.fld_stride + L.plane * oz];
            }
        }
    }
    store_padded(L, fld.eb, r, z, (TM)(eta_pref * s));
}

// grid (ceil(plane / 256), nz).  With a multiple of 8 chunks per layer the
// blocks go to the XCDs in y bands (xcd_band) rather than round-robin by row,
// so that the +-R rows a block reads sit in its own XCD's L2: 256^3 bulk 135 ->
// 130 us, and the contact values that read eta_bar next 141 -> 132 us.  The
// same order for the contact-value kernel itself gained nothing further.
template <int SIG, typename TM>
__global__ __launch_bounds__(256) void k_ballsum(LatticeDev L, double eta_pref, Fields<TM> fld,
                                                 const TM *__restrict__ rs)
{
    int z = (int)blockIdx.y, c = (int)blockIdx.x;
    if ((gridDim.x & 7) == 0) xcd_band((int)(blockIdx.x + gridDim.x * blockIdx.y), (int)gridDim.x, z, c);
    const int r = c * 256 + threadIdx.x;
    if (r < L.plane) d_ballsum<SIG>(L, eta_pref, fld, rs, z, r);
}

// ------------------------------------------ contact values at pair midpoints

// G slot b (bits x=1, y=2, z=4) at node r: g2 of the mean eta_bar over the
// nodes r + {0,1}^b, i.e. at the midpoint r + b/2 of every lattice pair whose
// offset has odd components exactly on the axes of b.
// The closure in FP64.  FP64 fields divide exactly; FP32 fields (which store
// the result rounded to FP32) take 1/(1-eta)^3 from a single-precision
// reciprocal refined by two Newton steps in FP64 (24 -> 48 -> full bits).
template <typename T>
__device__ __forceinline__ T g2_t(double eta, int model)
{
    const double om = 1.0 - eta;
    const double num = model ? (1.0 - 0.5 * eta) : (1.0 - 0.5 * eta + 0.25 * eta * eta);
    const double d = om * om * om;
    if constexpr (sizeof(T) == 8) {
        return num / d;
    } else {
        double r = (double)__builtin_amdgcn_rcpf((float)d);
        r = r * (2.0 - d * r);
        r = r * (2.0 - d * r);
        return (T)(num * r);
    }
}

#ifndef HSLB_NT_FIELD_MIB
#define HSLB_NT_FIELD_MIB 256
#endif
// Node r (0 <= r < plane) of layer z.  NT: non-temporal stores, for contact
// values that overflow the 256 MiB last-level cache on their own (256^3 bulk,
// 492 MB: this kernel 154 -> 139 us and the collide that reads them 1515 ->
// 1489 us).  Below that the collide loses from it: 6 us of 39 on the 64x64x136
// slit (17 MB), 15 us of 336 on the 128x128x264 slit (128 MB).
// The value of v held by the lane of node x + 1 (periodic), for lanes along
// whole x-rows: ROT 1 a wave per row of 64 nodes (wave_rol:1), ROT 2 a 16-lane
// row per row of 16 nodes (row_ror:15).  A DPP move, no memory access.
template <int ROT, typename TM>
__device__ __forceinline__ TM lane_xp1(TM v)
{
    static_assert(ROT == 1 || ROT == 2, "lane_xp1");
    constexpr int ctrl = ROT == 1 ? 0x134 : 0x12F;
    if constexpr (sizeof(TM) == 4) {
        return __builtin_bit_cast(TM, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, v),
                                                                  __builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
    } else {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned long long lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)b, (int)(uint32_t)b, ctrl,
                                                                            0xF, 0xF, false);
        const unsigned long long hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(b >> 32),
                                                                            (int)(uint32_t)(b >> 32), ctrl, 0xF, 0xF,
                                                                            false);
        return __builtin_bit_cast(TM, lo | (hi << 32));
    }
}

// ROT (see lane_xp1): the three eta_bar values at x + 1 come from the
// neighbouring lane's loads at x; every lane of a row must be active.
template <typename TM, bool NT = false, int ROT = 0>
__device__ __forceinline__ void d_gfield(const LatticeDev &L, int model, const Fields<TM> &fld, int z, int r)
{
    const int y = r / L.nx;
    const int x = r - y * L.nx;
    const int x1 = wrapc<1>(x, L.nx), y1 = wrapc<1>(y, L.ny);
    const int zp = z + L.hz;
    auto e = [&](int xx, int yy, int zz) -> double { return (double)fld.eb[xx + L.nx * (yy + L.ny * zz)]; };
    double e000, e100, e010, e001, e110, e101, e011;
    if constexpr (ROT != 0) {
        auto t = [&](int xx, int yy, int zz) -> TM { return fld.eb[xx + L.nx * (yy + L.ny * zz)]; };
        const TM t000 = t(x, y, zp), t010 = t(x, y1, zp), t001 = t(x, y, zp + 1);
        e000 = (double)t000;
        e010 = (double)t010;
        e001 = (double)t001;
        e011 = e(x, y1, zp + 1);
        e100 = (double)lane_xp1<ROT>(t000);
        e110 = (double)lane_xp1<ROT>(t010);
        e101 = (double)lane_xp1<ROT>(t001);
    } else {
        e000 = e(x, y, zp);
        e100 = e(x1, y, zp);
        e010 = e(x, y1, zp);
        e001 = e(x, y, zp + 1);
        e110 = e(x1, y1, zp);
        e101 = e(x1, y, zp + 1);
        e011 = e(x, y1, zp + 1);
    }
    const size_t fs = L.fld_stride;
    const double h = 0.5, q = 0.25;
    auto st = [&](TM *dst, TM v) {
        if constexpr (NT)
            store_padded_nt(L, dst, r, z, v);
        else
            store_padded(L, dst, r, z, v);
    };
    st(fld.G + 0 * fs, g2_t<TM>(e000, model));
    st(fld.G + 1 * fs, g2_t<TM>(h * (e000 + e100), model));
    st(fld.G + 2 * fs, g2_t<TM>(h * (e000 + e010), model));
    st(fld.G + 3 * fs, g2_t<TM>(q * ((e000 + e100) + (e010 + e110)), model));
    st(fld.G + 4 * fs, g2_t<TM>(h * (e000 + e001), model));
    st(fld.G + 5 * fs, g2_t<TM>(q * ((e000 + e100) + (e001 + e101)), model));
    st(fld.G + 6 * fs, g2_t<TM>(q * ((e000 + e010) + (e001 + e011)), model));
}

// grid (ceil(plane / 256), nz)
template <typename TM, bool NT, int ROT = 0>
__global__ __launch_bounds__(256) void k_gfield(LatticeDev L, int model, Fields<TM> fld)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < L.plane) d_gfield<TM, NT, ROT>(L, model, fld, (int)blockIdx.y, r);
}

// ------------------------------------------------------------ shell force

template <typename TC>
struct NodeCtx {
    int x, y, zp;
    TC u[3];
    TC ckap;  // chi(z) * kappa
};

// Byte offset, inside its layer, of the node at x + D (xb) or of the row at
// y + D (yb), periodic in x and y, for elements of ES bytes.  Offsets inside a
// layer fit 32 bits; the layer and field-slot parts are added to the base
// pointer, so that a block with uniform z keeps them in scalar registers and a
// shell read costs one vector add.
template <int D, int ES>
__device__ __forceinline__ uint32_t xb(int x, int nx)
{
    return (uint32_t)wrapc<D>(x, nx) * (uint32_t)ES;
}
template <int D, int ES>
__device__ __forceinline__ uint32_t yb(int y, int ny, int nx)
{
    return __umul24((uint32_t)wrapc<D>(y, ny), (uint32_t)nx * (uint32_t)ES);
}

// s.j of a loaded (n, jx, jy, jz) for the unit direction with components
// (SX, SY, SZ) in {-1, 0, 1} (not yet scaled by 1/sqrt(2) on a diagonal).
template <int SX, int SY, int SZ, typename TM, typename TC>
__device__ __forceinline__ TC s_dot_j(const TM q[4])
{
    if constexpr (SX != 0) {
        TC s = TC(SX) * (TC)q[1];
        if constexpr (SY != 0) s += TC(SY) * (TC)q[2];
        if constexpr (SZ != 0) s += TC(SZ) * (TC)q[3];
        return s;
    } else if constexpr (SY != 0) {
        TC s = TC(SY) * (TC)q[2];
        if constexpr (SZ != 0) s += TC(SZ) * (TC)q[3];
        return s;
    } else {
        return TC(SZ) * (TC)q[3];
    }
}

// The contact values G+ (midpoint of (r, r+d)) and G- (midpoint of (r, r-d))
// of one mirrored lattice pair, addressed as load_pair does.
template <int DX, int DY, int DZ, bool LZ, typename TM>
__device__ __forceinline__ void load_gpair(const Fields<TM> &F, const LatticeDev &L, int x, int y, int zp, TM &Gp,
                                           TM &Gm)
{
    constexpr int SLOT = (DX & 1) | ((DY & 1) << 1) | ((DZ & 1) << 2);
    constexpr int BXP = floordiv2(DX), BYP = floordiv2(DY), BZP = floordiv2(DZ);
    constexpr int BXM = floordiv2(-DX), BYM = floordiv2(-DY), BZM = floordiv2(-DZ);
    if constexpr (LZ) {
        constexpr int GB = (int)sizeof(TM);
        const size_t lay = (size_t)L.plane;
        const char *gs = (const char *)F.G + GB * (size_t)SLOT * L.fld_stride;
        const char *gzp = gs + GB * lay * (size_t)(zp + BZP);
        const char *gzm = gs + GB * lay * (size_t)(zp + BZM);
        Gp = *(const TM *)(gzp + (xb<BXP, GB>(x, L.nx) + yb<BYP, GB>(y, L.ny, L.nx)));
        Gm = *(const TM *)(gzm + (xb<BXM, GB>(x, L.nx) + yb<BYM, GB>(y, L.ny, L.nx)));
    } else {
        const size_t fs = L.fld_stride;
        const int gp = wrapc<BXP>(x, L.nx) + L.nx * (wrapc<BYP>(y, L.ny) + L.ny * (zp + BZP));
        const int gm = wrapc<BXM>(x, L.nx) + L.nx * (wrapc<BYM>(y, L.ny) + L.ny * (zp + BZM));
        Gp = F.G[SLOT * fs + gp];
        Gm = F.G[SLOT * fs + gm];
    }
}

// The (n, j) of r + (DX, DY, DZ), addressed as load_pair does.
template <int DX, int DY, int DZ, bool LZ, typename TM>
__device__ __forceinline__ void load_nj(const Fields<TM> &F, const LatticeDev &L, int x, int y, int zp, TM q[4])
{
    if constexpr (LZ) {
        constexpr int NJB = 4 * (int)sizeof(TM);
        const char *nz = (const char *)F.nj + NJB * (size_t)L.plane * (size_t)(zp + DZ);
        load4((const TM *)(nz + (xb<DX, NJB>(x, L.nx) + yb<DY, NJB>(y, L.ny, L.nx))), q);
    } else {
        load4(F.nj + 4 * (size_t)(wrapc<DX>(x, L.nx) + L.nx * (wrapc<DY>(y, L.ny) + L.ny * (zp + DZ))), q);
    }
}

// Loads of one mirrored lattice pair: the contact values G+ (midpoint of
// (r, r+d)) and G- (midpoint of (r, r-d)) and the (n, j) of r+d and r-d.
template <int DX, int DY, int DZ, bool LZ, typename TM>
__device__ __forceinline__ void load_pair(const Fields<TM> &F, const LatticeDev &L, int x, int y, int zp, TM &Gp,
                                          TM &Gm, TM qp[4], TM qm[4])
{
    load_gpair<DX, DY, DZ, LZ>(F, L, x, y, zp, Gp, Gm);
    if constexpr (LZ) {
        constexpr int NJB = 4 * (int)sizeof(TM);  // bytes of one (n, j) entry
        const size_t lay = (size_t)L.plane;
        const char *njp = (const char *)F.nj + NJB * lay * (size_t)(zp + DZ);
        const char *njm = (const char *)F.nj + NJB * lay * (size_t)(zp - DZ);
        load4((const TM *)(njp + (xb<DX, NJB>(x, L.nx) + yb<DY, NJB>(y, L.ny, L.nx))), qp);
        load4((const TM *)(njm + (xb<-DX, NJB>(x, L.nx) + yb<-DY, NJB>(y, L.ny, L.nx))), qm);
    } else {
        const int ip = wrapc<DX>(x, L.nx) + L.nx * (wrapc<DY>(y, L.ny) + L.ny * (zp + DZ));
        const int im = wrapc<-DX>(x, L.nx) + L.nx * (wrapc<-DY>(y, L.ny) + L.ny * (zp - DZ));
        load4(F.nj + 4 * (size_t)ip, qp);
        load4(F.nj + 4 * (size_t)im, qm);
    }
}

// The contact values G+ and G- of the pair with offset (DX, DY, DZ) from global
// memory, addressed as load_pair does for a block of uniform z.
template <int DX, int DY, int DZ>
__device__ __forceinline__ void load_g(const Fields<float> &F, const LatticeDev &L, int x, int y, int zp, float &Gp,
                                       float &Gm)
{
    constexpr int SLOT = (DX & 1) | ((DY & 1) << 1) | ((DZ & 1) << 2);
    constexpr int GB = (int)sizeof(float);
    const size_t lay = (size_t)L.plane;
    const char *gs = (const char *)F.G + GB * (size_t)SLOT * L.fld_stride;
    const char *gzp = gs + GB * lay * (size_t)(zp + floordiv2(DZ));
    const char *gzm = gs + GB * lay * (size_t)(zp + floordiv2(-DZ));
    Gp = *(const float *)(gzp + (xb<floordiv2(DX), GB>(x, L.nx) + yb<floordiv2(DY), GB>(y, L.ny, L.nx)));
    Gm = *(const float *)(gzm + (xb<floordiv2(-DX), GB>(x, L.nx) + yb<floordiv2(-DY), GB>(y, L.ny, L.nx)));
}

// x-neighbour exchange between the lanes of a wave (DPP moves between the
// lanes' registers, no memory access), for lanes laid out along whole periodic
// x-rows.  ROT 1: a wave is one x-row of 64 nodes (nx = 64); ROT 2: each
// 16-lane DPP row of the wave is one x-row of 16 nodes (nx = 16); ROT 3: an
// x-row of 128 or 256 nodes spans 2 or 4 waves of the block (the wave rotation
// of ROT 1, whose row-edge lanes then take the neighbouring wave's value, see
// s_xedge).  DIR +1 returns the value held by the lane of node x+1, DIR -1 that
// of node x-1, both periodic in x.  Every lane of a row must be active.
template <int ROT, int DIR>
__device__ __forceinline__ uint32_t lane_x(uint32_t v)
{
    static_assert((ROT >= 1 && ROT <= 3) && (DIR == 1 || DIR == -1), "lane_x");
    // wave_rol:1 / wave_ror:1 (lane l reads lane l+1 / l-1 mod 64); row_ror:15 /
    // row_ror:1 (lane l reads lane l+1 / l-1 mod 16 within its row)
    constexpr int ctrl = ROT != 2 ? (DIR > 0 ? 0x134 : 0x13C) : (DIR > 0 ? 0x12F : 0x121);
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, ctrl, 0xF, 0xF, false);
}
template <int ROT, int DIR, typename TM>
__device__ __forceinline__ void lane_x4(const TM src[4], TM dst[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if constexpr (sizeof(TM) == 4) {
            dst[k] = __builtin_bit_cast(TM, lane_x<ROT, DIR>(__builtin_bit_cast(uint32_t, src[k])));
        } else {
            const unsigned long long b = __builtin_bit_cast(unsigned long long, src[k]);
            const unsigned long long lo = lane_x<ROT, DIR>((uint32_t)b);
            const unsigned long long hi = lane_x<ROT, DIR>((uint32_t)(b >> 32));
            dst[k] = __builtin_bit_cast(TM, lo | (hi << 32));
        }
    }
}

// ROT 2 only: the value held by the lane of node x + K (periodic, |K| < 16) of
// the same 16-lane row (row_ror:N makes lane l read lane l - N mod 16).
template <int K, typename TM>
__device__ __forceinline__ TM lane_xk(TM v)
{
    constexpr int N = ((-K) % 16 + 16) % 16;
    if constexpr (N == 0) {
        return v;
    } else {
        static_assert(sizeof(TM) == 4, "lane_xk: 32-bit values");
        return __builtin_bit_cast(
            TM, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, v), __builtin_bit_cast(int, v), 0x120 + N, 0xF, 0xF,
                                            false));
    }
}
template <int K, typename TM>
__device__ __forceinline__ void lane_xk4(const TM src[4], TM dst[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = lane_xk<K>(src[k]);
}

// Difference of the two elements of one mirrored lattice pair, the corner d of
// direction q and the corner -d of direction -q:
//   e+ - e- = G+ [n+ - chi kappa s.(j+ - n+ u)] - G- [n- + chi kappa s.(j- - n- u)]
// with G+- the contact value at the midpoint of (r, r+-d).  The density part is
// written as ((G+ + G-)(n+ - n-) + (G+ - G-)(n+ + n-))/2, whose differences are
// exact in floating point for neighbouring values, so that the result keeps
// full relative precision even in FP32 although the two elements nearly
// cancel.  `su` is s.u(r) (s scaled by 1/sqrt(2) on the face diagonals).
//
// LZ: z is uniform over the block (layer-indexed grids); the layer parts of
// the addresses then stay scalar.  Grids with a per-lane z (batch, k_force)
// form one 32-bit node index per read instead, which needs fewer registers.
template <int SX, int SY, int SZ, bool DIAG, typename TM, typename TC>
__device__ __forceinline__ TC pair_math(TM gp, TM gm, const TM qp[4], const TM qm[4], const NodeCtx<TC> &c, TC su)
{
    const TC Gp = (TC)gp, Gm = (TC)gm;
    const TC np = (TC)qp[0], nm = (TC)qm[0];
    TC sjp = s_dot_j<SX, SY, SZ, TM, TC>(qp);
    TC sjm = s_dot_j<SX, SY, SZ, TM, TC>(qm);
    if constexpr (DIAG) {
        sjp *= TC(0.70710678118654752440);
        sjm *= TC(0.70710678118654752440);
    }
    const TC cp = sjp - np * su;
    const TC cm = sjm - nm * su;
    const TC dens = TC(0.5) * ((Gp + Gm) * (np - nm) + (Gp - Gm) * (np + nm));
    return dens - c.ckap * (Gp * cp + Gm * cm);
}

template <int DX, int DY, int DZ, int SX, int SY, int SZ, bool DIAG, bool LZ, typename TM, typename TC>
__device__ __forceinline__ TC pair_element(const Fields<TM> &F, const LatticeDev &L, const NodeCtx<TC> &c,
                                           TC su)
{
    TM gp, gm, qp[4], qm[4];
    load_pair<DX, DY, DZ, LZ>(F, L, c.x, c.y, c.zp, gp, gm, qp, qm);
    return pair_math<SX, SY, SZ, DIAG>(gp, gm, qp, qm, c, su);
}

// Offsets of corner (LA, LB) of the face diagonal with signs (SA, SB) in plane
// PL (0: xy, 1: xz, 2: yz).
template <int PL, int SA, int SB, int LA, int LB>
struct Diag {
    static constexpr int a = SA * LA, b = SB * LB;
    static constexpr int DX = (PL == 2) ? 0 : a;
    static constexpr int DY = (PL == 0) ? b : ((PL == 2) ? a : 0);
    static constexpr int DZ = (PL == 0) ? 0 : b;
    static constexpr int SX = (PL == 2) ? 0 : SA;
    static constexpr int SY = (PL == 0) ? SB : ((PL == 2) ? SA : 0);
    static constexpr int SZ = (PL == 0) ? 0 : SB;
};

// ROT 3: before the shell sum, lane 0 of each wave stores the (n, j) at r + d of
// the 8 shared corners d (those of the face diagonals of the xy and xz planes
// whose x-neighbour corner takes its reads from the lanes) and lane 63 the (n, j)
// at r - d; after the rotation, the row-edge lane takes the neighbouring wave's
// entry.  Layout [corner][0: lane 0 at r + d, 1: lane 63 at r - d][wave].
__shared__ float4 s_xedge[8 * 2 * 4];

template <int DX, int DY, int DZ, int EI>
__device__ __forceinline__ void xedge_one(const Fields<float> &F, const LatticeDev &L, int x, int y, int zp, int lane,
                                          int w)
{
    if (lane == 0 || lane == 63) {
        const int ip = wrapc<DX>(x, L.nx) + L.nx * (wrapc<DY>(y, L.ny) + L.ny * (zp + DZ));
        const int im = wrapc<-DX>(x, L.nx) + L.nx * (wrapc<-DY>(y, L.ny) + L.ny * (zp - DZ));
        const float4 q = *(const float4 *)(F.nj + 4 * (size_t)(lane == 0 ? ip : im));
        s_xedge[(EI * 2 + (lane == 0 ? 0 : 1)) * 4 + w] = q;
    }
}

// Fills s_xedge for the block; every thread of the block calls it, and a
// barrier must follow before the shell sum reads the entries.
template <int SIG>
__device__ __forceinline__ void xedge_prepass(const Fields<float> &F, const LatticeDev &L, int x, int y, int zp)
{
    constexpr int LL = ell_of(SIG);
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    // corner index as diag_pair numbers it: (plane * 2 + (SB < 0)) * 2 + (0: (l, l), 1: (l, l+1))
#define HSLB_XE(PL, SB, K)                                                                                    \
    xedge_one<Diag<PL, 1, SB, LL, LL + K>::DX, Diag<PL, 1, SB, LL, LL + K>::DY, Diag<PL, 1, SB, LL, LL + K>::DZ, \
              (PL * 2 + (SB > 0 ? 0 : 1)) * 2 + K>(F, L, x, y, zp, lane, w)
    HSLB_XE(0, 1, 0);
    HSLB_XE(0, 1, 1);
    HSLB_XE(0, -1, 0);
    HSLB_XE(0, -1, 1);
    HSLB_XE(1, 1, 0);
    HSLB_XE(1, 1, 1);
    HSLB_XE(1, -1, 0);
    HSLB_XE(1, -1, 1);
#undef HSLB_XE
}

// Pair elements read from global memory (the padded fields, any field type).
// ROT (see lane_x): the (n, j) of a face-diagonal corner whose x offset is one
// further than another corner's comes from the neighbouring lane's load of
// that corner, the same values; 0: every element loads its own.
template <bool LZ, typename TM, int ROT_ = 0>
struct GlobalShell {
    static constexpr int ROT = ROT_;
    const Fields<TM> &F;
    const LatticeDev &L;
    template <int DX, int DY, int DZ, int SX, int SY, int SZ, bool DIAG, typename TC>
    __device__ __forceinline__ TC elem(const NodeCtx<TC> &c, TC su) const
    {
        return pair_element<DX, DY, DZ, SX, SY, SZ, DIAG, LZ>(F, L, c, su);
    }
    // The element of corner d = (DX, DY, DZ) and, in *e_next, that of corner
    // d + (SA, 0, 0): its (n, j) at r + d + SA e_x is the (n, j) at r' + d of
    // the node r' = r + SA e_x, and its (n, j) at r - d - SA e_x that at r'' - d
    // of r'' = r - SA e_x.  EI: the corner's index in s_xedge (ROT 3).
    template <int DX, int DY, int DZ, int SX, int SY, int SZ, int SA, int EI, typename TC>
    __device__ __forceinline__ TC elem_share(const NodeCtx<TC> &c, TC su, TC &e_next) const
    {
        static_assert(ROT != 0, "elem_share needs lanes along x-rows");
        TM gp, gm, qp[4], qm[4];
        load_pair<DX, DY, DZ, LZ>(F, L, c.x, c.y, c.zp, gp, gm, qp, qm);
        const TC e = pair_math<SX, SY, SZ, true>(gp, gm, qp, qm, c, su);
        TM hp, hm, rp[4], rm[4];
        load_gpair<DX + SA, DY, DZ, LZ>(F, L, c.x, c.y, c.zp, hp, hm);
        lane_x4<ROT, SA>(qp, rp);
        lane_x4<ROT, -SA>(qm, rm);
        if constexpr (ROT == 3) {
            static_assert(SA == 1 && sizeof(TM) == 4, "row-edge exchange: FP32 fields, corners moved by +x");
            const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
            const int wr = L.nx >> 6, wb = w - w % wr;  // waves per x-row, first wave of this row
            const int wn = wb + (w - wb + 1) % wr, wp = wb + (w - wb + wr - 1) % wr;
            const float4 ep = s_xedge[(EI * 2 + 0) * 4 + wn];
            const float4 em = s_xedge[(EI * 2 + 1) * 4 + wp];
            const bool hi = lane == 63, lo = lane == 0;
            rp[0] = hi ? ep.x : rp[0];
            rp[1] = hi ? ep.y : rp[1];
            rp[2] = hi ? ep.z : rp[2];
            rp[3] = hi ? ep.w : rp[3];
            rm[0] = lo ? em.x : rm[0];
            rm[1] = lo ? em.y : rm[1];
            rm[2] = lo ? em.z : rm[2];
            rm[3] = lo ? em.w : rm[3];
        }
        e_next = pair_math<SX, SY, SZ, true>(hp, hm, rp, rm, c, su);
        return e;
    }
};

// The interpolated quadrature point q = (SA, SB) in plane PL and its mirror -q:
// W s_q sum_k alpha_k (e+_k - e-_k), k over the four bilinear corners.
template <int PL, int SA, int SB, int LL, typename SRC, typename TC>
__device__ __forceinline__ void diag_pair(const SRC &src, const NodeCtx<TC> &c, const TC *alpha, TC S[3])
{
    constexpr int A = (PL == 2) ? 1 : 0;
    constexpr int B = (PL == 0) ? 1 : 2;
    using D00 = Diag<PL, SA, SB, LL, LL>;
    using D01 = Diag<PL, SA, SB, LL, LL + 1>;
    using D10 = Diag<PL, SA, SB, LL + 1, LL>;
    using D11 = Diag<PL, SA, SB, LL + 1, LL + 1>;
    const TC su = TC(0.70710678118654752440) * (TC(SA) * c.u[A] + TC(SB) * c.u[B]);
    TC d;
    if constexpr (SRC::ROT != 0 && PL != 2) {
        // corners (l+1, .) are corners (l, .) moved by SA along x
        static_assert(D10::DX == D00::DX + SA && D11::DX == D01::DX + SA, "x-neighbour corners");
        TC e10, e11;
        constexpr int EI = (PL * 2 + (SB > 0 ? 0 : 1)) * 2;
        const TC e00 = src.template elem_share<D00::DX, D00::DY, D00::DZ, D00::SX, D00::SY, D00::SZ, SA, EI>(c, su, e10);
        const TC e01 =
            src.template elem_share<D01::DX, D01::DY, D01::DZ, D01::SX, D01::SY, D01::SZ, SA, EI + 1>(c, su, e11);
        d = alpha[0] * e00;
        d += alpha[1] * e01;
        d += alpha[2] * e10;
        d += alpha[3] * e11;
    } else {
        d = alpha[0] * src.template elem<D00::DX, D00::DY, D00::DZ, D00::SX, D00::SY, D00::SZ, true>(c, su);
        d += alpha[1] * src.template elem<D01::DX, D01::DY, D01::DZ, D01::SX, D01::SY, D01::SZ, true>(c, su);
        d += alpha[2] * src.template elem<D10::DX, D10::DY, D10::DZ, D10::SX, D10::SY, D10::SZ, true>(c, su);
        d += alpha[3] * src.template elem<D11::DX, D11::DY, D11::DZ, D11::SX, D11::SY, D11::SZ, true>(c, su);
    }
    const TC w = TC((1.0 / 15.0) * 0.70710678118654752440) * d;
    S[A] += TC(SA) * w;
    S[B] += TC(SB) * w;
}

// Both face-diagonal quadrature points (1, 1) and (1, -1) of plane PL (0: xy,
// 1: xz) for lanes along 16-node x-rows (ROT 2): the same sums as
// diag_pair<PL, 1, 1> followed by diag_pair<PL, 1, -1>, with every value that
// another lane of the row loads taken from that lane.  With b the offset off
// the x axis and LA, LB in {l, l+1}:
//  - (n, j): per LB, P at r + (l, LB) and M at r - (l, LB) are loaded; the other
//    corners' entries lie on the same two rows, 1, 2l or 2l+1 nodes away in x;
//  - contact values: per corner d = (LA, LB) of the point (1, 1), G+ and G- are
//    loaded; the corner (LA, -LB) of the point (1, -1) finds its G- at the
//    same row as G+(d), LA nodes back in x, and its G+ with G-(d), LA ahead.
template <int PL, int LL, bool LZ, typename TM, typename TC>
__device__ __forceinline__ void diag_plane16(const Fields<TM> &F, const LatticeDev &L, const NodeCtx<TC> &c,
                                             const TC *alpha, TC S[3])
{
    static_assert(PL == 0 || PL == 1, "x-planes only");
    constexpr int B = (PL == 0) ? 1 : 2;
    TC e[2][2][2];  // [0: point (1, 1), 1: point (1, -1)][LA - l][LB - l]
    const TC sup = TC(0.70710678118654752440) * (c.u[0] + c.u[B]);
    const TC sum = TC(0.70710678118654752440) * (c.u[0] - c.u[B]);
#define HSLB_D16_LB(KB)                                                                                        \
    {                                                                                                          \
        using Q0 = Diag<PL, 1, 1, LL, LL + KB>;                                                                \
        TM P[4], M[4];                                                                                         \
        load_nj<Q0::DX, Q0::DY, Q0::DZ, LZ>(F, L, c.x, c.y, c.zp, P);                                          \
        load_nj<-Q0::DX, -Q0::DY, -Q0::DZ, LZ>(F, L, c.x, c.y, c.zp, M);                                       \
        HSLB_D16_LA(0, KB)                                                                                     \
        HSLB_D16_LA(1, KB)                                                                                     \
    }
#define HSLB_D16_LA(KA, KB)                                                                                    \
    {                                                                                                          \
        using Q = Diag<PL, 1, 1, LL + KA, LL + KB>;                                                            \
        using R = Diag<PL, 1, -1, LL + KA, LL + KB>;                                                           \
        constexpr int LA = LL + KA;                                                                            \
        TM gp, gm, qp[4], qm[4], rp[4], rm[4];                                                                 \
        load_gpair<Q::DX, Q::DY, Q::DZ, LZ>(F, L, c.x, c.y, c.zp, gp, gm);                                     \
        lane_xk4<KA>(P, qp);                                                                                   \
        lane_xk4<-KA>(M, qm);                                                                                  \
        e[0][KA][KB] = pair_math<Q::SX, Q::SY, Q::SZ, true>(gp, gm, qp, qm, c, sup);                          \
        lane_xk4<LL + LA>(M, rp);                                                                              \
        lane_xk4<-(LL + LA)>(P, rm);                                                                           \
        e[1][KA][KB] = pair_math<R::SX, R::SY, R::SZ, true>(lane_xk<LA>(gm), lane_xk<-LA>(gp), rp, rm, c, sum); \
    }
    HSLB_D16_LB(0)
    HSLB_D16_LB(1)
#undef HSLB_D16_LA
#undef HSLB_D16_LB
    const TC wq = TC((1.0 / 15.0) * 0.70710678118654752440);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        TC d = alpha[0] * e[k][0][0];
        d += alpha[1] * e[k][0][1];
        d += alpha[2] * e[k][1][0];
        d += alpha[3] * e[k][1][1];
        const TC w = wq * d;
        S[0] += w;
        S[B] += k == 0 ? w : -w;
    }
}

// S = sum_q W_q s_q sum_k alpha_qk G_qk [ ... ] over the 18-point rule, with
// directions taken in (q, -q) pairs (a uniform fluid at rest gives exactly 0).
template <int SIG, bool LZ, typename TM, typename TC, int ROT = 0>
__device__ __forceinline__ void shell_sum(const Fields<TM> &F, const LatticeDev &L, const NodeCtx<TC> &c,
                                          const TC *alpha, TC S[3])
{
    constexpr int LL = ell_of(SIG);
    const GlobalShell<LZ, TM, ROT> src{F, L};
    const TC w30 = TC(1.0 / 30.0);
    S[0] = w30 * pair_element<SIG, 0, 0, 1, 0, 0, false, LZ>(F, L, c, c.u[0]);
    S[1] = w30 * pair_element<0, SIG, 0, 0, 1, 0, false, LZ>(F, L, c, c.u[1]);
    S[2] = w30 * pair_element<0, 0, SIG, 0, 0, 1, false, LZ>(F, L, c, c.u[2]);
    if constexpr (ROT == 2) {
        diag_plane16<0, LL, LZ>(F, L, c, alpha, S);
        diag_plane16<1, LL, LZ>(F, L, c, alpha, S);
    } else {
        diag_pair<0, 1, 1, LL>(src, c, alpha, S);
        diag_pair<0, 1, -1, LL>(src, c, alpha, S);
        diag_pair<1, 1, 1, LL>(src, c, alpha, S);
        diag_pair<1, 1, -1, LL>(src, c, alpha, S);
    }
    diag_pair<2, 1, 1, LL>(src, c, alpha, S);
    diag_pair<2, 1, -1, LL>(src, c, alpha, S);
}

// ------------------------------------- shell sum staged through LDS (FP32 fields)
//
// A block of 256 threads owns a 64 x 4 tile of one layer (a wave per row, so
// the population accesses stay whole rows).  The shell reads of neighbouring
// nodes overlap: an (n, j) entry of the layer is read by up to 20 nodes of the
// tile, one of the layers z -+ l, z -+ (l + 1) by up to 4 through the face
// diagonals of the xz plane.  The block copies those regions of the shell
// fields into LDS once, with global-to-LDS loads issued together with the
// population loads (their latency overlaps the moment sums):
//   A   layer z: (n, j) over the tile widened by sigma in x and y (the pairs
//       along x and y, the face diagonals of the xy plane) and contact-value
//       slots 0..3 widened by GH;
//   B   layers z -+ (l + 1), z -+ l: (n, j) widened by l + 1 in x (face
//       diagonals of the xz plane), optionally the 8 contact-value planes
//       they read (STAGE_BG).
// The pair along z and the face diagonals of the yz plane, whose reads a
// 4-row tile hardly shares, read global memory.  The elements are summed in
// the order of shell_sum with the same arithmetic, so the force is bit for bit
// that of the direct reads.  The halo of a 64 x 4 tile is large (phase A copies
// 4.75 entries per node of the tile), and the copies cost about what the
// gathers they replace cost: the kernel is an option, not the default.
namespace stage {
constexpr int TX = 64, TY = 4;  // tile
constexpr int GH = 4;           // contact-value halo: |floor(d / 2)| <= 4 for sigma <= 8
constexpr int GWX = TX + 2 * GH;
static_assert(GWX % 4 == 0 && GH % 4 == 0, "contact-value rows are copied as float4");
static_assert(TX * TY == 256, "a block of 256 threads per tile");

// Which contact values go through LDS (phase A, phase B); the others are read
// from global memory like the pair along z.  Measured on the 256^3 bulk
// (sigma 6): staging both needs 61 KB of LDS per block (two blocks per compute
// unit) and takes 1764 us per collide; staging neither, 2035 us; phase A's
// only (52 KB, three blocks), 1554 us, the best of the three.
constexpr bool STAGE_AG = true, STAGE_BG = false;

template <int SIG>
struct Geo {
    static_assert(SIG >= 2 && SIG <= 8, "staged shell sum covers sigma 2..8");
    static constexpr int LL = ell_of(SIG);
    static constexpr int H1 = LL + 1;
    static constexpr int AWX = TX + 2 * SIG, AWY = TY + 2 * SIG;  // phase A (n, j) region
    static constexpr int AGY = TY + 2 * GH;                         // phase A contact-value rows
    static constexpr int BWX = TX + 2 * H1;                         // phase B (n, j) rows
    static constexpr int A_NJ = AWX * AWY;                          // float4 entries
    static constexpr int B_NJ = 4 * BWX * TY;
    static constexpr int A_G4 = STAGE_AG ? 4 * AGY * (GWX / 4) : 0;  // float4 entries
    static constexpr int B_G4 = STAGE_BG ? 8 * TY * (GWX / 4) : 0;
    // one LDS array of float4: A (n, j), B (n, j), A contact values, B contact values
    static constexpr int O_BNJ = A_NJ, O_AG = A_NJ + B_NJ, O_BG = O_AG + A_G4;
    static constexpr int SIZE = O_BG + B_G4;
    // layer offsets of phase B, indexed -(l+1), -l, l, l+1
    __host__ __device__ static constexpr int zi(int dz)
    {
        return dz == -H1 ? 0 : (dz == -LL ? 1 : (dz == LL ? 2 : 3));
    }
    __host__ __device__ static constexpr int dz_of(int i)
    {
        return i == 0 ? -H1 : (i == 1 ? -LL : (i == 2 ? LL : H1));
    }
};
// the largest contact-value offset, floor(-sigma / 2), stays inside the halo
static_assert(floordiv2(-8) >= -GH && floordiv2(8) <= GH, "contact-value halo");

struct Tile {
    float4 *lds;  // Geo<SIG>::SIZE entries
    int x0, y0;   // tile origin
    int lx, ly;   // this node inside the tile
};

// Global-to-LDS load of 16 bytes per lane: lane l of the wave writes LDS
// entry `wave_base` + l (wave_base is uniform over the wave).
__device__ __forceinline__ void to_lds(const float4 *src, float4 *wave_base)
{
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                     (__attribute__((address_space(3))) void *)wave_base, 16, 0, 0);
}

// Entries [0, CNT) of a region, entry i from src_of(i): the wave issuing
// entries [256 k + 64 w, 256 k + 64 w + 64) writes them to dst + that range.
template <int CNT, typename F>
__device__ __forceinline__ void copy_region(float4 *dst, F src_of)
{
    const int w64 = __builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63;
#pragma unroll
    for (int k = 0; k < (CNT + 255) / 256; ++k) {
        const int i = (int)threadIdx.x + 256 * k;
        if (i < CNT) to_lds(src_of(i), dst + 256 * k + w64);
    }
}

// Issues the copies of phases A and B for the tile of layer zp (padded index).
template <int SIG>
__device__ __forceinline__ void copy_tile(const Fields<float> &F, const LatticeDev &L, const Tile &t, int zp)
{
    using G = Geo<SIG>;
    const float4 *nj = (const float4 *)F.nj;
    const size_t pl = (size_t)L.plane;
    // A (n, j): [x0 - SIG, x0 + TX + SIG) x [y0 - SIG, y0 + TY + SIG) of layer zp
    copy_region<G::A_NJ>(t.lds, [&](int i) {
        const int ry = i / G::AWX, rx = i - ry * G::AWX;
        const int gx = wrapr(t.x0 + rx - SIG, L.nx), gy = wrapr(t.y0 + ry - SIG, L.ny);
        return nj + pl * (size_t)zp + (gx + L.nx * gy);
    });
    // B (n, j): layers zp + dz_of(p), [x0 - H1, x0 + TX + H1) x [y0, y0 + TY)
    copy_region<G::B_NJ>(t.lds + G::O_BNJ, [&](int i) {
        const int p = i / (G::BWX * TY), rem = i - p * (G::BWX * TY);
        const int ry = rem / G::BWX, rx = rem - ry * G::BWX;
        const int gx = wrapr(t.x0 + rx - G::H1, L.nx);
        return nj + pl * (size_t)(zp + G::dz_of(p)) + (gx + L.nx * (t.y0 + ry));
    });
    // A contact values: slots 0..3 of layer zp, [x0 - GH, x0 + TX + GH) x [y0 - GH, y0 + TY + GH)
    constexpr int R4 = GWX / 4;
    if constexpr (STAGE_AG) copy_region<G::A_G4>(t.lds + G::O_AG, [&](int i) {
        const int slot = i / (G::AGY * R4), rem = i - slot * (G::AGY * R4);
        const int ry = rem / R4, c4 = rem - ry * R4;
        const int gx = wrapr(t.x0 - GH + 4 * c4, L.nx), gy = wrapr(t.y0 + ry - GH, L.ny);
        return (const float4 *)(F.G + (size_t)slot * L.fld_stride + pl * (size_t)zp + (gx + L.nx * gy));
    });
    // B contact values: plane c = (layer offset p, x parity b) = 2 p + b holds slot
    // b | (dz & 1) << 2 of layer zp + floor(dz / 2), [x0 - GH, x0 + TX + GH) x [y0, y0 + TY)
    if constexpr (STAGE_BG) copy_region<G::B_G4>(t.lds + G::O_BG, [&](int i) {
        const int c = i / (TY * R4), rem = i - c * (TY * R4);
        const int ry = rem / R4, c4 = rem - ry * R4;
        const int dz = G::dz_of(c >> 1);
        const int slot = (c & 1) | ((dz & 1) << 2);
        const int gx = wrapr(t.x0 - GH + 4 * c4, L.nx);
        return (const float4 *)(F.G + (size_t)slot * L.fld_stride + pl * (size_t)(zp + floordiv2(dz)) +
                                (gx + L.nx * (t.y0 + ry)));
    });
}

// Pair elements read from the staged regions of phase PH (0: A, 1: B).
template <int SIG, int PH>
struct StagedShell {
    static constexpr int ROT = 0;
    const Tile &t;
    const Fields<float> &F;
    const LatticeDev &L;
    template <int DX, int DY, int DZ, int SX, int SY, int SZ, bool DIAG, typename TC>
    __device__ __forceinline__ TC elem(const NodeCtx<TC> &c, TC su) const
    {
        using G = Geo<SIG>;
        const float *g = (const float *)t.lds;
        float4 a, b;
        float gp, gm;
        if constexpr (PH == 0) {
            static_assert(DZ == 0, "phase A holds layer z");
            constexpr int slot = (DX & 1) | ((DY & 1) << 1);
            const int o = t.ly * G::AWX + t.lx;
            a = t.lds[o + (DY + SIG) * G::AWX + DX + SIG];
            b = t.lds[o + (SIG - DY) * G::AWX + SIG - DX];
            if constexpr (STAGE_AG) {
                const int og = 4 * G::O_AG + slot * G::AGY * GWX + t.ly * GWX + t.lx;
                gp = g[og + (floordiv2(DY) + GH) * GWX + floordiv2(DX) + GH];
                gm = g[og + (floordiv2(-DY) + GH) * GWX + floordiv2(-DX) + GH];
            } else {
                load_g<DX, DY, DZ>(F, L, c.x, c.y, c.zp, gp, gm);
            }
        } else {
            static_assert(DY == 0, "phase B holds the xz diagonals");
            constexpr int cp = 2 * G::zi(DZ) + (DX & 1), cm = 2 * G::zi(-DZ) + (DX & 1);
            const int o = G::O_BNJ + t.ly * G::BWX + t.lx + G::H1;
            a = t.lds[o + G::zi(DZ) * G::BWX * TY + DX];
            b = t.lds[o + G::zi(-DZ) * G::BWX * TY - DX];
            if constexpr (STAGE_BG) {
                const int og = 4 * G::O_BG + t.ly * GWX + t.lx + GH;
                gp = g[og + cp * TY * GWX + floordiv2(DX)];
                gm = g[og + cm * TY * GWX + floordiv2(-DX)];
            } else {
                load_g<DX, DY, DZ>(F, L, c.x, c.y, c.zp, gp, gm);
            }
        }
        const float qp[4] = {a.x, a.y, a.z, a.w}, qm[4] = {b.x, b.y, b.z, b.w};
        return pair_math<SX, SY, SZ, DIAG>(gp, gm, qp, qm, c, su);
    }
};

}  // namespace stage

// shell_sum with the pairs of layer z and the face diagonals of the xz plane
// read from the LDS regions that copy_tile filled; every thread of the block
// calls it (it waits for the copies and synchronises the block).
template <int SIG, typename TC>
__device__ __forceinline__ void shell_sum_staged(const Fields<float> &F, const LatticeDev &L, const NodeCtx<TC> &c,
                                                 const TC *alpha, TC S[3], const stage::Tile &t)
{
    constexpr int LL = ell_of(SIG);
    const TC w30 = TC(1.0 / 30.0);
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's global-to-LDS loads
    __syncthreads();
    const stage::StagedShell<SIG, 0> a{t, F, L};
    const stage::StagedShell<SIG, 1> b{t, F, L};
    const GlobalShell<true, float> direct{F, L};
    S[0] = w30 * a.template elem<SIG, 0, 0, 1, 0, 0, false>(c, c.u[0]);
    S[1] = w30 * a.template elem<0, SIG, 0, 0, 1, 0, false>(c, c.u[1]);
    S[2] = w30 * pair_element<0, 0, SIG, 0, 0, 1, false, true>(F, L, c, c.u[2]);
    diag_pair<0, 1, 1, LL>(a, c, alpha, S);
    diag_pair<0, 1, -1, LL>(a, c, alpha, S);
    diag_pair<1, 1, 1, LL>(b, c, alpha, S);
    diag_pair<1, 1, -1, LL>(b, c, alpha, S);
    diag_pair<2, 1, 1, LL>(direct, c, alpha, S);
    diag_pair<2, 1, -1, LL>(direct, c, alpha, S);
}

// Mean-field attraction at a fluid node: -n times the central difference of
// phi; the neighbours of a fluid node lie inside the array (walls are >= 1 layer).
__device__ __forceinline__ void att_force(const LatticeDev &L, const StepConst &sc, int x, int y, int z, double n,
                                          double Fa[3])
{
    int zu = z + 1, zd = z - 1;
    if (L.zper) {
        zu = (zu == L.nz) ? 0 : zu;
        zd = (zd < 0) ? L.nz - 1 : zd;
    }
    const double *P = sc.phi;
    const int row = L.nx * (y + L.ny * z);
    Fa[0] = -n * (P[wrapc<1>(x, L.nx) + row] - P[wrapc<-1>(x, L.nx) + row]) / 2.0;
    Fa[1] = -n * (P[x + L.nx * (wrapc<1>(y, L.ny) + L.ny * z)] - P[x + L.nx * (wrapc<-1>(y, L.ny) + L.ny * z)]) / 2.0;
    Fa[2] = -n * (P[x + L.nx * (y + L.ny * zu)] - P[x + L.nx * (y + L.ny * zd)]) / 2.0;
}

// Total force C^(1) + n g at a fluid node with local moments (n, u).
// STAGED: the shell sum reads LDS through the block's tile *tile (FP32 fields;
// every thread of the block must call).
template <int SIG, bool LZ, typename TM, bool MASK = true, bool STAGED = false, int ROT = 0>
__device__ __forceinline__ void node_force(const Fields<TM> &F, const LatticeDev &L, const StepConst &sc,
                                           const double *__restrict__ chi, int x, int y, int z, double n,
                                           const double u[3], double Fo[3], const stage::Tile *tile = nullptr)
{
#if HSLB_FORCE_FP64
    using TC = double;
#else
    using TC = TM;
#endif
    if constexpr (SIG == 0) {
        // interaction force supplied per node (learned force and its correction)
        const int id = x + L.nx * (y + L.ny * z);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double c1 = 0.0;
            if (sc.fext) c1 += sc.fscale * (double)sc.fext[(size_t)a * L.N + id];
            if (sc.fdelta) c1 += (double)sc.fdelta[(size_t)a * L.N + id];
            Fo[a] = c1 + n * sc.g[a];
        }
        return;
    } else {
    TC S[3] = {TC(0), TC(0), TC(0)};
    if (sc.hs_on) {
        NodeCtx<TC> c;
        c.x = x;
        c.y = y;
        c.zp = z + L.hz;
        c.u[0] = (TC)u[0];
        c.u[1] = (TC)u[1];
        c.u[2] = (TC)u[2];
        if constexpr (MASK)
            c.ckap = (TC)((sc.chi_n ? sc.chi_n[x + L.nx * (y + L.ny * z)] : chi[z]) * sc.kappa);
        else
            c.ckap = (TC)(chi[z] * sc.kappa);
        const TC alpha[4] = {(TC)sc.alpha[0], (TC)sc.alpha[1], (TC)sc.alpha[2], (TC)sc.alpha[3]};
        if constexpr (STAGED)
            shell_sum_staged<SIG>(F, L, c, alpha, S, *tile);
        else
            shell_sum<SIG, LZ, TM, TC, ROT>(F, L, c, alpha, S);
    }
    double Fa[3] = {0.0, 0.0, 0.0};
    if (sc.phi) att_force(L, sc, x, y, z, n, Fa);
    const double pn = sc.pref * n;
    Fo[0] = pn * (double)S[0] + Fa[0] + n * sc.g[0];
    Fo[1] = pn * (double)S[1] + Fa[1] + n * sc.g[1];
    Fo[2] = pn * (double)S[2] + Fa[2] + n * sc.g[2];
    }
}

// ------------------------------------------------- collide and stream

// Node r (0 <= r < plane) of fluid layer z.  STAGED: the shell sum goes
// through the LDS tile *tile (see shell_sum_staged).  ROT: lanes along whole
// x-rows share x-neighbour (n, j) reads (see GlobalShell).
template <int SIG, bool LZ, typename TF, typename TM, bool MASK = false, bool NT = false, bool STAGED = false,
          int ROT = 0>
__device__ __forceinline__ void d_collide(const LatticeDev &L, const StepConst &sc, const double *__restrict__ chi,
                                          const TF *__restrict__ fin, TF *__restrict__ fout, const Fields<TM> &fld,
                                          int z, int r, const stage::Tile *tile = nullptr)
{
    const int y = r / L.nx;
    const int x = r - y * L.nx;

    // LZ: byte offsets with the direction and layer parts on the base
    // pointers and the node's place in its layer as a 32-bit lane offset;
    // otherwise node indices
    constexpr uint32_t EB = sizeof(TF);
    const size_t dstride = EB * (size_t)L.pop_stride;
    const size_t lstride = EB * (size_t)L.plane;
    const uint32_t rb = (uint32_t)r * EB;
    const int id = z * L.plane + r;
    // solid mask: a solid node only restates its (zero) populations against
    // the write reference; its neighbours bounce off it
    uint32_t lk = 0;
    if (MASK && sc.links) {
        lk = sc.links[id];
        if (lk & LINK_SOLID) {
            const double *rw = layer_ref(sc.nref_w, z);
#pragma unroll
            for (int i = 0; i < NQ; ++i) fout[(size_t)i * L.pop_stride + id] = (TF)(0.0 - rw[i]);
            return;
        }
    }
    // the stored values are kept through the shell sum (half the registers of
    // FP64 populations) and turned into FP64 populations again for the collision
    TF fs[NQ];
    const double *rr = layer_ref(sc.nref_r, z);
    if constexpr (LZ) {
        const char *fz = (const char *)fin + lstride * (size_t)z;
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const TF *p = (const TF *)(fz + dstride * i + rb);
            if constexpr (NT)
                fs[i] = __builtin_nontemporal_load(p);
            else
                fs[i] = *p;
        }
    } else if constexpr (NT) {
#pragma unroll
        for (int i = 0; i < NQ; ++i) fs[i] = __builtin_nontemporal_load(fin + (size_t)i * L.pop_stride + id);
    } else {
#pragma unroll
        for (int i = 0; i < NQ; ++i) fs[i] = fin[(size_t)i * L.pop_stride + id];
    }
    // the staged shell fields load into LDS while the moments are summed
    if constexpr (STAGED) stage::copy_tile<SIG>(fld, L, *tile, z + L.hz);
    double n = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const double fi = (double)fs[i] + rr[i];
        n += fi;
        if (CX[i] > 0) jx += fi;
        if (CX[i] < 0) jx -= fi;
        if (CY[i] > 0) jy += fi;
        if (CY[i] < 0) jy -= fi;
        if (CZ[i] > 0) jz += fi;
        if (CZ[i] < 0) jz -= fi;
    }
    const double inv_n = (n != 0.0) ? 1.0 / n : 0.0;
    const double u[3] = {jx * inv_n, jy * inv_n, jz * inv_n};
    double Fv[3];
    node_force<SIG, LZ, TM, MASK, STAGED, ROT>(fld, L, sc, chi, x, y, z, n, u, Fv, tile);

    // BGK relaxation (10) towards the equilibrium (11), with the first-order
    // source, for opposite velocities i and i + 1 together: with cu = c_i.u,
    // f_eq = w n (1 - 1.5 u.u + 4.5 cu^2) +- 3 w n cu and the source
    // +- 3 w c_i.F; f - f_eq is formed in FP64.
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double omega = 1.0 / sc.tau;
    const double base = 1.0 - 1.5 * uu;
    double f[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i] = (double)fs[i] + rr[i];
    double fq[NQ];
    fq[0] = f[0] - omega * (f[0] - (1.0 / 3.0) * n * base);
#pragma unroll
    for (int i = 1; i < NQ; i += 2) {
        const double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        const double cF = CX[i] * Fv[0] + CY[i] * Fv[1] + CZ[i] * Fv[2];
        const double wn = wq(i) * n;
        const double A = wn * fma(4.5 * cu, cu, base);
        const double B = (3.0 * wn) * cu;
        const double src = (3.0 * wq(i)) * cF;
        fq[i] = fma(-omega, f[i] - (A + B), f[i] + src);
        fq[i + 1] = fma(-omega, f[i + 1] - (A - B), f[i + 1] - src);
    }
    // The write references of the layers the populations land in, read before
    // the first store: later reads could not be scalar (the compiler cannot
    // rule out that the stores alias the table) and would each wait out a
    // vector-memory round trip.
    int zu = z + 1, zd = z - 1;
    if (L.zper) {
        zu = (zu == L.nz) ? 0 : zu;
        zd = (zd < 0) ? L.nz - 1 : zd;
    } else {
        zu = (zu < L.nz) ? zu : z;   // a fluid layer's upper neighbour exists in a slit
        zd = (zd >= 0) ? zd : z;
    }
    const double *rwz = layer_ref(sc.nref_w, z), *rwu = layer_ref(sc.nref_w, zu), *rwd = layer_ref(sc.nref_w, zd);
    double rwh[NQ], rwl[NQ];  // layer z; the layer direction i lands in
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        rwh[i] = rwz[i];
        rwl[i] = CZ[i] > 0 ? rwu[i] : (CZ[i] < 0 ? rwd[i] : rwh[i]);
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const double fp = fq[i];
        const int xt = wrapr(x + CX[i], L.nx);
        const int yt = wrapr(y + CY[i], L.ny);
        int zt = z + CZ[i];
        bool bounce = (lk >> i) & 1u;
        if (L.zper) {
            zt = (zt < 0) ? zt + L.nz : ((zt >= L.nz) ? zt - L.nz : zt);
        } else {
            bounce = bounce || (zt < L.wall_lo) || (zt >= L.nz - L.wall_hi);
        }
        // stored relative to the reference of the layer it lands in
        const TF vb = (TF)(fp - rwh[OPP[i]]);
        const TF vs = (TF)(fp - rwl[i]);
        if constexpr (LZ) {
            char *fo = (char *)fout;
            if (bounce) {
                TF *p = (TF *)(fo + dstride * OPP[i] + lstride * (size_t)z + rb);
                if constexpr (NT)
                    __builtin_nontemporal_store(vb, p);
                else
                    *p = vb;
            } else {
                TF *p = (TF *)(fo + dstride * i + lstride * (size_t)zt +
                               ((uint32_t)xt * EB + __umul24((uint32_t)yt, (uint32_t)L.nx * EB)));
                if constexpr (NT)
                    __builtin_nontemporal_store(vs, p);
                else
                    *p = vs;
            }
        } else if constexpr (NT) {
            if (bounce)
                __builtin_nontemporal_store(vb, fout + (size_t)OPP[i] * L.pop_stride + id);
            else
                __builtin_nontemporal_store(vs, fout + (size_t)i * L.pop_stride + xt + L.nx * (yt + L.ny * zt));
        } else {
            if (bounce)
                fout[(size_t)OPP[i] * L.pop_stride + id] = vb;
            else
                fout[(size_t)i * L.pop_stride + xt + L.nx * (yt + L.ny * zt)] = vs;
        }
    }
}

// Waves per SIMD the collide kernel is compiled for (register budget
// 512 / waves).  3 leaves the compiler its natural ~130 VGPRs; 4 and 5
// (104 and 96 VGPRs, no spills) measured 25 % slower: the shell reads of more
// resident waves overflow the L1.
#ifndef HSLB_COLLIDE_WAVES
#define HSLB_COLLIDE_WAVES 3
#endif

// 1-D grid over (layer, chunk of 256 nodes of the layer): z is uniform over a
// block, so the rows of the storage reference tables come in through scalar
// loads.  band: blocks go to the XCDs by xcd_band (each XCD sweeps one eighth
// of every layer, all layers together) instead of xcd_block (each XCD sweeps
// whole layers of its own z slab).  MASK: the solid-mask code is compiled in (a
// separate instance, so that the plain path keeps its registers).
// NT: populations loaded and stored non-temporally, for lattices whose two
// population copies overflow the last-level cache (256^3 bulk: 1603 -> 1539 us);
// the cache-resident benchmark slit gains nothing from it.  That instance also
// addresses its reads by 32-bit node indices (as the batch kernel does) rather
// than by layer-uniform base offsets: 1513 against 1530 us on the bulk, while
// the slit keeps the layer-uniform form (39.5 against 40.8 us).
template <int SIG, typename TF, typename TM, bool MASK, bool NT, int ROT>
__global__ __launch_bounds__(256, HSLB_COLLIDE_WAVES) void k_collide(LatticeDev L, StepConst sc, const double *__restrict__ chi,
                                                 const TF *__restrict__ fin, TF *__restrict__ fout,
                                                 Fields<TM> fld, int cpp, int band)
{
    int zl, c;
    if (band) {
        xcd_band((int)blockIdx.x, cpp, zl, c);
    } else {
        const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);
        zl = lb / cpp;
        c = lb - zl * cpp;
    }
    const int r = c * 256 + threadIdx.x;
    const int z = (L.zper ? 0 : L.wall_lo) + zl;
    if constexpr (ROT == 3 && SIG >= 2) {
        // the host takes ROT 3 only for a plane that is a multiple of 256 nodes:
        // every thread of the block is a node and reaches the barrier
        const int y = r / L.nx;
        xedge_prepass<SIG>(fld, L, r - y * L.nx, y, z + L.hz);
        __syncthreads();
    }
    if (r < L.plane) d_collide<SIG, !NT, TF, TM, MASK, NT, false, ROT>(L, sc, chi, fin, fout, fld, z, r);
}

// k_collide for FP32 storage and fields with the shell sum staged through LDS:
// one block per 64 x 4 tile of a fluid layer (nx a multiple of 64, ny of 4, no
// solid mask, hard-sphere force on, sigma 2..8); blocks in (layer, tile row,
// tile) order, spread over the XCDs as k_collide's.  Up to 59 KB of LDS per
// block: three blocks per compute unit for sigma <= 6, two above.
template <int SIG, bool NT>
__global__ __launch_bounds__(256, 3) void k_collide_tiles(LatticeDev L, StepConst sc, const double *__restrict__ chi,
                                                          const float *__restrict__ fin, float *__restrict__ fout,
                                                          Fields<float> fld)
{
    __shared__ float4 s_lds[stage::Geo<SIG>::SIZE];
    const int tnx = L.nx / stage::TX;
    const int tpl = tnx * (L.ny / stage::TY);
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int zl = lb / tpl;
    const int tl = lb - zl * tpl;
    const int ty = tl / tnx;
    stage::Tile tile;
    tile.lds = s_lds;
    tile.x0 = (tl - ty * tnx) * stage::TX;
    tile.y0 = ty * stage::TY;
    tile.lx = (int)threadIdx.x % stage::TX;
    tile.ly = (int)threadIdx.x / stage::TX;
    const int r = (tile.y0 + tile.ly) * L.nx + tile.x0 + tile.lx;
    const int z = (L.zper ? 0 : L.wall_lo) + zl;
    d_collide<SIG, true, float, float, false, NT, true>(L, sc, chi, fin, fout, fld, z, r, &tile);
}

template <int SIG, typename TF, typename TM>
__global__ __launch_bounds__(256) void k_force(LatticeDev L, StepConst sc, const double *__restrict__ chi,
                                               const TF *__restrict__ fin, Fields<TM> fld, double *__restrict__ Fout)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    const int z = id / L.plane;
    const int rem = id - z * L.plane;
    const int y = rem / L.nx;
    const int x = rem - y * L.nx;
    double Fv[3] = {0.0, 0.0, 0.0};
    if (is_fluid_z(L, z)) {
        double n = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        const double *rr = layer_ref(sc.nref_r, z);
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const double fi = (double)fin[(size_t)i * L.pop_stride + id] + rr[i];
            n += fi;
            jx += CX[i] * fi;
            jy += CY[i] * fi;
            jz += CZ[i] * fi;
        }
        const double inv_n = (n != 0.0) ? 1.0 / n : 0.0;
        const double u[3] = {jx * inv_n, jy * inv_n, jz * inv_n};
        node_force<SIG, false>(fld, L, sc, chi, x, y, z, n, u, Fv);
    }
    Fout[id] = Fv[0];
    Fout[L.N + id] = Fv[1];
    Fout[2 * (size_t)L.N + id] = Fv[2];
}

// ------------------------------------------------- mean-field attraction

// Pass along x of the padded density field: a = sum_m w[m] n(x + m - R).
// grid (ceil(plane / 256), nz); R may exceed nx (the offsets wrap again).
// ROT (see lane_xp1): one load of n(x - R), each further tap from the
// neighbouring lane, in the same order.
template <typename TM, int ROT = 0>
__global__ __launch_bounds__(256) void k_att_x(LatticeDev L, AttWeights aw, const TM *__restrict__ n,
                                               double *__restrict__ out)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int z = (int)blockIdx.y;
    if (r >= L.plane) return;
    const int y = r / L.nx;
    const int x = r - y * L.nx;
    const TM *row = n + (size_t)L.plane * (z + L.hz) + (size_t)L.nx * y;
    int xm = (x - aw.R) % L.nx;
    xm = xm < 0 ? xm + L.nx : xm;
    double s = 0.0;
    if constexpr (ROT != 0) {
        TM v = row[xm];
#pragma unroll 8
        for (int m = 0; m <= 2 * aw.R; ++m) {
            s += aw.w[m] * (double)v;
            v = lane_xp1<ROT>(v);
        }
    } else {
#pragma unroll 8
        for (int m = 0; m <= 2 * aw.R; ++m) {
            s += aw.w[m] * (double)row[xm];
            xm = (xm + 1 == L.nx) ? 0 : xm + 1;
        }
    }
    out[(size_t)L.plane * z + r] = s;
}

// Pass along y: b = sum_m w[m] a(y + m - R).
__global__ __launch_bounds__(256) void k_att_y(LatticeDev L, AttWeights aw, const double *__restrict__ a,
                                               double *__restrict__ out)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int z = (int)blockIdx.y;
    if (r >= L.plane) return;
    const int y = r / L.nx;
    const int x = r - y * L.nx;
    const double *col = a + (size_t)L.plane * z + x;
    int ym = (y - aw.R) % L.ny;
    ym = ym < 0 ? ym + L.ny : ym;
    double s = 0.0;
#pragma unroll 8
    for (int m = 0; m <= 2 * aw.R; ++m) {
        s += aw.w[m] * col[(size_t)L.nx * ym];
        ym = (ym + 1 == L.ny) ? 0 : ym + 1;
    }
    out[(size_t)L.plane * z + r] = s;
}

// Pass along z: phi = -eps sum_m w[m] b(z + m - R), wrapping for a periodic z
// axis and with nothing beyond the array otherwise.
__global__ __launch_bounds__(256) void k_att_z(LatticeDev L, AttWeights aw, const double *__restrict__ b,
                                               double *__restrict__ out)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int z = (int)blockIdx.y;
    if (r >= L.plane) return;
    double s = 0.0;
    if (L.zper) {
        int zm = (z - aw.R) % L.nz;
        zm = zm < 0 ? zm + L.nz : zm;
#pragma unroll 8
        for (int m = 0; m <= 2 * aw.R; ++m) {
            s += aw.w[m] * b[(size_t)L.plane * zm + r];
            zm = (zm + 1 == L.nz) ? 0 : zm + 1;
        }
    } else {
        // only the offsets that stay inside the array contribute
        const int m0 = max(0, aw.R - z), m1 = min(2 * aw.R, L.nz - 1 - z + aw.R);
#pragma unroll 8
        for (int m = m0; m <= m1; ++m) s += aw.w[m] * b[(size_t)L.plane * (z + m - aw.R) + r];
    }
    out[(size_t)L.plane * z + r] = -aw.eps * s;
}

// -------------------------------------------------------------- reductions

// Layer profiles from FP64 sums taken straight from the populations:
// out[0][z] = mean n over the layer, out[1+a][z] = (sum j_a)/(sum n),
// out[4][z] = sum n.  One block per layer, fixed summation order.
template <typename TF>
__global__ __launch_bounds__(256) void k_profiles(LatticeDev L, const double *__restrict__ nref,
                                                  const TF *__restrict__ f, double *__restrict__ out)
{
    const int z = blockIdx.x;
    __shared__ double red[4][4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (is_fluid_z(L, z)) {
        const double *rr = layer_ref(nref, z);
        for (int r = threadIdx.x; r < L.plane; r += 256) {
            const int id = z * L.plane + r;
            double n = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const double fi = (double)f[(size_t)i * L.pop_stride + id] + rr[i];
                n += fi;
                jx += CX[i] * fi;
                jy += CY[i] * fi;
                jz += CZ[i] * fi;
            }
            s[0] += n;
            s[1] += jx;
            s[2] += jy;
            s[3] += jz;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = wave_sum(s[k]);
        if (lane == 0) red[wv][k] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
        out[z] = t[0] / (double)L.plane;
#pragma unroll
        for (int a = 0; a < 3; ++a) out[(1 + a) * L.nz + z] = (t[0] != 0.0) ? t[1 + a] / t[0] : 0.0;
        out[4 * L.nz + z] = t[0];
    }
}

template <typename TM>
__global__ __launch_bounds__(256) void k_unpad(LatticeDev L, const TM *__restrict__ src, double *__restrict__ dst)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    const int z = id / L.plane;
    const int rem = id - z * L.plane;
    dst[id] = (double)src[rem + L.plane * (z + L.hz)];
}

// Moments for export: n and u = j/n in FP64 from the populations.
template <typename TF>
__global__ __launch_bounds__(256) void k_export_moments(LatticeDev L, const double *__restrict__ nref,
                                                        const TF *__restrict__ f, double *__restrict__ n_out,
                                                        double *__restrict__ u_out)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    double n = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    if (is_fluid_z(L, id / L.plane)) {
        const double *rr = layer_ref(nref, id / L.plane);
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const double fi = (double)f[(size_t)i * L.pop_stride + id] + rr[i];
            n += fi;
            jx += CX[i] * fi;
            jy += CY[i] * fi;
            jz += CZ[i] * fi;
        }
    }
    const double inv = (n != 0.0) ? 1.0 / n : 0.0;
    n_out[id] = n;
    u_out[id] = jx * inv;
    u_out[L.N + id] = jy * inv;
    u_out[2 * (size_t)L.N + id] = jz * inv;
}

template <typename TF>
__global__ __launch_bounds__(256) void k_get_pop(LatticeDev L, const double *__restrict__ nref,
                                                 const TF *__restrict__ f, double *__restrict__ out)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    const int z = id / L.plane;
    const bool fl = is_fluid_z(L, z);
    const double *r = layer_ref(nref, z);
#pragma unroll
    for (int i = 0; i < NQ; ++i)
        out[(size_t)i * L.N + id] = fl ? (double)f[(size_t)i * L.pop_stride + id] + r[i] : 0.0;
}

template <typename TF>
__global__ __launch_bounds__(256) void k_set_pop(LatticeDev L, const double *__restrict__ nref,
                                                 const double *__restrict__ in, TF *__restrict__ f)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    const int z = id / L.plane;
    const bool fl = is_fluid_z(L, z);
    const double *r = layer_ref(nref, z);
#pragma unroll
    for (int i = 0; i < NQ; ++i)
        f[(size_t)i * L.pop_stride + id] = fl ? (TF)(in[(size_t)i * L.N + id] - r[i]) : (TF)0;
}


// ------------------------------------------------------- batched ensemble

template <typename TM>
__device__ __forceinline__ Fields<TM> shift_fields(const Fields<TM> &F, int off)
{
    Fields<TM> g;
    g.n = F.n + off;
    g.nj = F.nj + 4 * (size_t)off;
    g.eb = F.eb + off;
    g.G = F.G + off;
    return g;
}

// Collision at fluid index k of a slit (fluid nodes counted from the first
// fluid layer); the layer is computed per lane (see kb_phase).
template <int SIG, int ROT, typename TF, typename TM>
__device__ __forceinline__ void batch_collide(const LatticeDev &L, const StepConst &sc, const double *__restrict__ chi,
                                              const TF *__restrict__ fin, TF *__restrict__ fout,
                                              const Fields<TM> &fld, int k)
{
    const int first = L.zper ? 0 : L.wall_lo * L.plane;
    const int last = L.zper ? L.N : (L.nz - L.wall_hi) * L.plane;
    const int id = first + k;
    if (id >= last) return;
    const int z = id / L.plane;
    // The ensemble's populations (about 700 MB for 512 slits) overflow the
    // last-level cache: they stream non-temporally so that the shell fields stay
    // cached (6366 -> 6597 MLUPS).
    d_collide<SIG, false, TF, TM, false, true, false, ROT>(L, sc, chi, fin, fout, fld, z, id - z * L.plane);
}

// Collide phase of every slit in one persistent launch: the grid walks the
// fluid work items; each item's descriptor (and sigma, hence the shell
// stencil) is uniform over the block.  A kernel of its own, so that the
// lighter phases of kb_phase keep a small register budget.  ROT 2: every slit
// is 16 nodes wide in x, so that each 16-lane row of a wave is one x-row and
// the shell sum shares x-neighbour (n, j) reads between lanes.
template <typename TF, typename TM, int ROT>
__global__ __launch_bounds__(256, HSLB_COLLIDE_WAVES) void kb_collide(const SlitDesc *__restrict__ desc,
                                                     const WorkItem *__restrict__ work, int nwork,
                                                     const TF *__restrict__ fin, TF *__restrict__ fout,
                                                     Fields<TM> fld, const double *__restrict__ chi)
{
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const WorkItem it = work[w];
        const SlitDesc &d = desc[it.slit];
        const Fields<TM> F = shift_fields(fld, d.fld_off);
        const TF *fi = fin + d.pop_off;
        TF *fo = fout + d.pop_off;
        const double *ch = chi + d.chi_off;
        const int idx = it.block * 256 + (int)threadIdx.x;
        switch (d.sigma) {
        case 2: batch_collide<2, ROT>(d.L, d.sc, ch, fi, fo, F, idx); break;
        case 3: batch_collide<3, ROT>(d.L, d.sc, ch, fi, fo, F, idx); break;
        case 4: batch_collide<4, ROT>(d.L, d.sc, ch, fi, fo, F, idx); break;
        case 5: batch_collide<5, ROT>(d.L, d.sc, ch, fi, fo, F, idx); break;
        case 6: batch_collide<6, ROT>(d.L, d.sc, ch, fi, fo, F, idx); break;
        case 7: batch_collide<7, ROT>(d.L, d.sc, ch, fi, fo, F, idx); break;
        case 8: batch_collide<8, ROT>(d.L, d.sc, ch, fi, fo, F, idx); break;
        default: break;
        }
    }
}

// Persistent kernel of one phase of the step for every slit: the grid walks
// the work list; each item is one block of 256 indices of one slit, whose
// descriptor (and sigma, hence the shell stencil) is uniform over the block.
// ROT 2: every slit is 16 nodes wide, and the contact values take their
// x + 1 eta_bar values from the neighbouring lane of the 16-lane row.
template <typename TF, typename TM, int ROT = 0>
__global__ __launch_bounds__(256) void kb_phase(int phase, const SlitDesc *__restrict__ desc,
                                                const WorkItem *__restrict__ work, int nwork,
                                                const TF *__restrict__ fin, TF *__restrict__ fout, Fields<TM> fld,
                                                TM *__restrict__ rs, const double *__restrict__ chi)
{
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
        const WorkItem it = work[w];
        const SlitDesc &d = desc[it.slit];
        const int idx = it.block * 256 + threadIdx.x;
        const Fields<TM> F = shift_fields(fld, d.fld_off);
        TM *rsl = rs + d.fld_off;
        const TF *fi = fin + d.pop_off;
        TF *fo = fout + d.pop_off;
        const double *ch = chi + d.chi_off;
        switch (phase) {
        case 0:
            // the layer is computed per lane: in this kernel scalar reads of
            // the reference rows would spill scalar registers
            if (idx < d.L.N) d_moments(d.L, d.sc.nref_r, fi, F, idx / d.L.plane, idx % d.L.plane);
            break;
        case 3:
            if (idx < d.L.N) d_gfield<TM, false, ROT>(d.L, d.sc.g2_model, F, idx / d.L.plane, idx % d.L.plane);
            break;
        case 4: {
            // phases 0 and 1 in one: every slit's layer is a whole number of
            // 256-node blocks of whole x-rows (the host checks), so the block
            // forms the row sums of its own densities, as k_moments_rs does;
            // the row sums of the padding stay the zeros they were set to
            __shared__ TM sn[256];
            const int z = idx / d.L.plane, r = idx - z * d.L.plane;
            sn[threadIdx.x] = d_moments(d.L, d.sc.nref_r, fi, F, z, r);
            __syncthreads();
            switch (d.sigma) {
            case 2: block_rowsums<2>(d.L, sn, rsl, z, r); break;
            case 3: block_rowsums<3>(d.L, sn, rsl, z, r); break;
            case 4: block_rowsums<4>(d.L, sn, rsl, z, r); break;
            case 5: block_rowsums<5>(d.L, sn, rsl, z, r); break;
            case 6: block_rowsums<6>(d.L, sn, rsl, z, r); break;
            case 7: block_rowsums<7>(d.L, sn, rsl, z, r); break;
            case 8: block_rowsums<8>(d.L, sn, rsl, z, r); break;
            default: break;
            }
            __syncthreads();  // sn is refilled by the next work item
            break;
        }
        default:
#define HSLB_BPH(SG)                                                                     \
    case SG:                                                                             \
        if (phase == 1) {                                                                \
            if (idx < d.L.plane * (d.L.nz + 2 * (SG / 2)))                               \
                d_rowsum<SG>(d.L, F, rsl, idx / d.L.plane, idx % d.L.plane);             \
        } else if (phase == 2) {                                                         \
            if (idx < d.L.N) d_ballsum<SG>(d.L, d.sc.eta_pref, F, rsl, idx / d.L.plane, idx % d.L.plane); \
        }                                                                                \
        break;
            switch (d.sigma) {
                HSLB_BPH(2)
                HSLB_BPH(3)
                HSLB_BPH(4)
                HSLB_BPH(5)
                HSLB_BPH(6)
                HSLB_BPH(7)
                HSLB_BPH(8)
            default: break;
            }
#undef HSLB_BPH
        }
    }
}

template <typename TF>
__global__ __launch_bounds__(256) void kb_profiles(const SlitDesc *__restrict__ desc, const WorkItem *__restrict__ items,
                                                   const int *__restrict__ prof_off, const TF *__restrict__ f,
                                                   double *__restrict__ out)
{
    const WorkItem it = items[blockIdx.x];
    const SlitDesc &d = desc[it.slit];
    const LatticeDev &L = d.L;
    const int z = it.block;
    const TF *fs = f + d.pop_off;
    __shared__ double red[4][4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (is_fluid_z(L, z)) {
        const double *rr = layer_ref(d.sc.nref_r, z);
        for (int r = threadIdx.x; r < L.plane; r += 256) {
            const int id = z * L.plane + r;
            double n = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const double fi = (double)fs[(size_t)i * L.pop_stride + id] + rr[i];
                n += fi;
                jx += CX[i] * fi;
                jy += CY[i] * fi;
                jz += CZ[i] * fi;
            }
            s[0] += n;
            s[1] += jx;
            s[2] += jy;
            s[3] += jz;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = wave_sum(s[k]);
        if (lane == 0) red[wv][k] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
        double *o = out + prof_off[it.slit];
        o[z] = t[0] / (double)L.plane;
#pragma unroll
        for (int a = 0; a < 3; ++a) o[(1 + a) * L.nz + z] = (t[0] != 0.0) ? t[1 + a] / t[0] : 0.0;
        o[4 * L.nz + z] = t[0];
    }
}

// Layer means of the stored populations of every slit: items (slit, z); the
// new reference goes to the write table.
template <typename TF>
__global__ __launch_bounds__(256) void kb_layer_means(const SlitDesc *__restrict__ desc,
                                                      const WorkItem *__restrict__ items, const TF *__restrict__ f)
{
    const WorkItem it = items[blockIdx.x];
    const SlitDesc &d = desc[it.slit];
    d_layer_means(d.L, f + d.pop_off, d.L.pop_stride, d.sc.nref_r, const_cast<double *>(d.sc.nref_w), it.block);
}

// Plain device-to-device copy (16-byte lanes, grid-stride): the achievable
// HBM bandwidth reference and the calibration kernel of the traffic counters.
__global__ __launch_bounds__(256) void k_round_f32(double *__restrict__ a, int count)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < count) a[k] = (double)(float)a[k];
}

__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) b[i] = a[i];
}

// ------------------------------------------------- 39-velocity lattice

// Third-order equilibrium of velocity I: w n [1 + xi + xi^2/2 - u^2/(2 s) +
// xi^3/6 - xi u^2/(2 s)], xi = c.u / s, s = v_T^2 = 2/3.
template <int I>
__device__ __forceinline__ double feq39_of(double n, const double u[3], double uu_s)
{
    constexpr double is = 1.0 / CS2_39;
    const double xi = (C39X[I] * u[0] + C39Y[I] * u[1] + C39Z[I] * u[2]) * is;
    return w39(I) * n * (1.0 + xi + 0.5 * xi * xi - 0.5 * uu_s + xi * xi * xi * (1.0 / 6.0) - 0.5 * xi * uu_s);
}

// Thermal: the Maxwellian at (n, u, T) through h^(3) about the lattice
// temperature s (xi = c/sqrt(s), u~ = u/sqrt(s), th1 = T/s - 1):
// w n [1 + xi.u~ + ((xi.u~)^2 - u~^2 + th1 (xi^2 - 3))/2
//      + (xi.u~)((xi.u~)^2 - 3 u~^2 + 3 th1 (xi^2 - 5))/6].  uu_s = u~^2.
template <int I>
__device__ __forceinline__ double feq39t_of(double n, const double u[3], double uu_s, double th1)
{
    constexpr double is = 1.0 / CS2_39;
    constexpr double xx = (C39X[I] * C39X[I] + C39Y[I] * C39Y[I] + C39Z[I] * C39Z[I]) * is;
    const double xu = (C39X[I] * u[0] + C39Y[I] * u[1] + C39Z[I] * u[2]) * is;
    return w39(I) * n *
           (1.0 + xu + 0.5 * (xu * xu - uu_s + th1 * (xx - 3.0)) +
            xu * (xu * xu - 3.0 * uu_s + 3.0 * th1 * (xx - 5.0)) * (1.0 / 6.0));
}

template <bool TH, int I>
__device__ __forceinline__ double feq39x(double n, const double u[3], double uu_s, double th1)
{
    if constexpr (TH)
        return feq39t_of<I>(n, u, uu_s, th1);
    else
        return feq39_of<I>(n, u, uu_s);
}

template <bool TH, int... I>
__device__ __forceinline__ void feq39_all(double n, const double u[3], double th1, double *out,
                                          std::integer_sequence<int, I...>)
{
    const double uu_s = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / CS2_39;
    ((out[I] = feq39x<TH, I>(n, u, uu_s, th1)), ...);
}

// T null: the lattice temperature (the isothermal equilibrium).
__global__ __launch_bounds__(256) void k_feq39(LatticeDev L, const double *__restrict__ n,
                                               const double *__restrict__ u, const double *__restrict__ T,
                                               double *__restrict__ out)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    double f[Q39];
    if (is_fluid_z(L, id / L.plane)) {
        const double uv[3] = {u[id], u[L.N + id], u[2 * (size_t)L.N + id]};
        if (T)
            feq39_all<true>(n[id], uv, T[id] / CS2_39 - 1.0, f, std::make_integer_sequence<int, Q39>{});
        else
            feq39_all<false>(n[id], uv, 0.0, f, std::make_integer_sequence<int, Q39>{});
    } else {
#pragma unroll
        for (int i = 0; i < Q39; ++i) f[i] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < Q39; ++i) out[(size_t)i * L.N + id] = f[i];
}

// n and j of a node from its 39 populations (0 on solid layers).
__device__ __forceinline__ void moments39(const LatticeDev &L, const double *__restrict__ f, size_t id, int z,
                                          double &n, double &jx, double &jy, double &jz)
{
    n = jx = jy = jz = 0.0;
    if (!is_fluid_z(L, z)) return;
#pragma unroll
    for (int i = 0; i < Q39; ++i) {
        const double fi = f[(size_t)i * L.pop_stride + id];
        n += fi;
        jx += C39X[i] * fi;
        jy += C39Y[i] * fi;
        jz += C39Z[i] * fi;
    }
}

// n, j and sum f c^2 of a node in one pass (0 on solid layers).
__device__ __forceinline__ void moments39e(const LatticeDev &L, const double *__restrict__ f, size_t id, int z,
                                           double &n, double &jx, double &jy, double &jz, double &e)
{
    n = jx = jy = jz = e = 0.0;
    if (!is_fluid_z(L, z)) return;
#pragma unroll
    for (int i = 0; i < Q39; ++i) {
        const double fi = f[(size_t)i * L.pop_stride + id];
        n += fi;
        jx += C39X[i] * fi;
        jy += C39Y[i] * fi;
        jz += C39Z[i] * fi;
        e += (double)(C39X[i] * C39X[i] + C39Y[i] * C39Y[i] + C39Z[i] * C39Z[i]) * fi;
    }
}

// Temperature from the moments: n T = (sum f c^2 - n u^2) / 3 (0 where n = 0).
__device__ __forceinline__ double temp_of(double n, double jx, double jy, double jz, double e)
{
    if (n == 0.0) return 0.0;
    const double inv = 1.0 / n;
    return (e * inv - (jx * jx + jy * jy + jz * jz) * inv * inv) / 3.0;
}

// grid (ceil(plane / 256), nz)
template <bool TH>
__global__ __launch_bounds__(256) void k_moments39(LatticeDev L, const double *__restrict__ f, Fields<double> fld)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int z = (int)blockIdx.y;
    if (r >= L.plane) return;
    double n, jx, jy, jz, e = 0.0;
    const size_t id = (size_t)z * L.plane + r;
    if constexpr (TH)
        moments39e(L, f, id, z, n, jx, jy, jz, e);
    else
        moments39(L, f, id, z, n, jx, jy, jz);
    store_padded(L, fld.n, r, z, n);
    store_padded4(L, fld.nj, r, z, n, jx, jy, jz);
    if constexpr (TH) store_padded(L, fld.T, r, z, temp_of(n, jx, jy, jz, e));
}

// Moments (and temperature) fused with the row sums of the two-pass ball sum,
// as k_moments_rs: the block holds whole x-rows of layer z.
template <int SIG, bool TH>
__global__ __launch_bounds__(256) void k_moments39_rs(LatticeDev L, const double *__restrict__ f, Fields<double> fld,
                                                      double *__restrict__ rs)
{
    __shared__ double sn[256];
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int z = (int)blockIdx.y;
    double n, jx, jy, jz, e = 0.0;
    const size_t id = (size_t)z * L.plane + r;
    if constexpr (TH)
        moments39e(L, f, id, z, n, jx, jy, jz, e);
    else
        moments39(L, f, id, z, n, jx, jy, jz);
    store_padded(L, fld.n, r, z, n);
    store_padded4(L, fld.nj, r, z, n, jx, jy, jz);
    if constexpr (TH) store_padded(L, fld.T, r, z, temp_of(n, jx, jy, jz, e));
    sn[threadIdx.x] = n;
    __syncthreads();
    block_rowsums<SIG>(L, sn, rs, z, r);
}

__global__ __launch_bounds__(256) void k_export39(LatticeDev L, const double *__restrict__ f, double *__restrict__ n,
                                                  double *__restrict__ u)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    double m, jx, jy, jz;
    moments39(L, f, id, id / L.plane, m, jx, jy, jz);
    const double inv = (m != 0.0) ? 1.0 / m : 0.0;
    n[id] = m;
    u[id] = jx * inv;
    u[L.N + id] = jy * inv;
    u[2 * (size_t)L.N + id] = jz * inv;
}

// Layer profiles as k_profiles: out[z] = mean n, out[(1 + a) nz + z] = u_a,
// out[4 nz + z] = sum n.  grid (nz)
__global__ __launch_bounds__(256) void k_profiles39(LatticeDev L, const double *__restrict__ f, double *__restrict__ out)
{
    const int z = blockIdx.x;
    __shared__ double red[4][4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = threadIdx.x; r < L.plane; r += 256) {
        double n, jx, jy, jz;
        moments39(L, f, (size_t)z * L.plane + r, z, n, jx, jy, jz);
        s[0] += n;
        s[1] += jx;
        s[2] += jy;
        s[3] += jz;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = wave_sum(s[k]);
        if (lane == 0) red[wv][k] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) t[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
        out[z] = t[0] / (double)L.plane;
#pragma unroll
        for (int a = 0; a < 3; ++a) out[(1 + a) * L.nz + z] = (t[0] != 0.0) ? t[1 + a] / t[0] : 0.0;
        out[4 * L.nz + z] = t[0];
    }
}

// Hermite coefficients of the non-equilibrium part d = f - f_eq:
// a2 = sum h2 d over (xx, yy, zz, xy, xz, yz), a3 = sum h3 d over
// (xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz), with
// h2_ab = c_a c_b - s d_ab and h3_abg = c_a c_b c_g - s (c_a d_bg + c_b d_ag + c_g d_ab).
template <int I>
__device__ __forceinline__ void herm_acc(double d, double a2[6], double a3[10])
{
    constexpr double s = CS2_39;
    constexpr double x = C39X[I], y = C39Y[I], z = C39Z[I];
    a2[0] += (x * x - s) * d;
    a2[1] += (y * y - s) * d;
    a2[2] += (z * z - s) * d;
    if constexpr (C39X[I] * C39Y[I] != 0) a2[3] += (x * y) * d;
    if constexpr (C39X[I] * C39Z[I] != 0) a2[4] += (x * z) * d;
    if constexpr (C39Y[I] * C39Z[I] != 0) a2[5] += (y * z) * d;
    if constexpr (C39X[I] != 0) a3[0] += (x * x * x - 3.0 * s * x) * d;
    if constexpr (C39Y[I] != 0) a3[1] += (y * y * y - 3.0 * s * y) * d;
    if constexpr (C39Z[I] != 0) a3[2] += (z * z * z - 3.0 * s * z) * d;
    if constexpr (C39Y[I] != 0) a3[3] += (x * x * y - s * y) * d;
    if constexpr (C39Z[I] != 0) a3[4] += (x * x * z - s * z) * d;
    if constexpr (C39X[I] != 0) a3[5] += (x * y * y - s * x) * d;
    if constexpr (C39Z[I] != 0) a3[6] += (y * y * z - s * z) * d;
    if constexpr (C39X[I] != 0) a3[7] += (x * z * z - s * x) * d;
    if constexpr (C39Y[I] != 0) a3[8] += (y * z * z - s * y) * d;
    if constexpr (C39X[I] * C39Y[I] * C39Z[I] != 0) a3[9] += (x * y * z) * d;
}

// The projection h2(c) : a2 / (2 s^2) + h3(c) : a3 / (6 s^3) as a cubic
// polynomial in c, P(c) = K0 + K1.c + c.K2.c + K3 : ccc, with
//   K0 = -tr a2 / (2 s),  K1_a = -(sum_b a3_abb) / (2 s^2),
//   K2_aa = a2_aa / (2 s^2), K2_ab = a2_ab / s^2 (a < b, both orders),
//   K3_aaa = a3_aaa / (6 s^3), K3_aab = a3_aab / (2 s^3) (three orders),
//   K3_xyz = a3_xyz / s^3 (six orders);
// k[] holds (K0, K1 x y z, K2 xx yy zz xy xz yz, K3 xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz).
__device__ __forceinline__ void proj_coeffs(const double a2[6], const double a3[10], double k[20])
{
    constexpr double s = CS2_39;
    constexpr double i2 = 1.0 / (2.0 * s * s), i3 = 1.0 / (s * s * s);
    k[0] = -(a2[0] + a2[1] + a2[2]) * (1.0 / (2.0 * s));
    k[1] = -(a3[0] + a3[5] + a3[7]) * i2;
    k[2] = -(a3[3] + a3[1] + a3[8]) * i2;
    k[3] = -(a3[4] + a3[6] + a3[2]) * i2;
    k[4] = a2[0] * i2;
    k[5] = a2[1] * i2;
    k[6] = a2[2] * i2;
    k[7] = a2[3] * (2.0 * i2);
    k[8] = a2[4] * (2.0 * i2);
    k[9] = a2[5] * (2.0 * i2);
#pragma unroll
    for (int m = 0; m < 3; ++m) k[10 + m] = a3[m] * (i3 / 6.0);
#pragma unroll
    for (int m = 3; m < 9; ++m) k[10 + m] = a3[m] * (i3 / 2.0);
    k[19] = a3[9] * i3;
}

template <int I>
__device__ __forceinline__ double proj_of(const double k[20])
{
    constexpr int x = C39X[I], y = C39Y[I], z = C39Z[I];
    double p = k[0];
    if constexpr (x != 0) p += x * k[1] + (x * x) * k[4] + (x * x * x) * k[10];
    if constexpr (y != 0) p += y * k[2] + (y * y) * k[5] + (y * y * y) * k[11];
    if constexpr (z != 0) p += z * k[3] + (z * z) * k[6] + (z * z * z) * k[12];
    if constexpr (x * y != 0) p += (x * y) * k[7] + (x * x * y) * k[13] + (x * y * y) * k[15];
    if constexpr (x * z != 0) p += (x * z) * k[8] + (x * x * z) * k[14] + (x * z * z) * k[17];
    if constexpr (y * z != 0) p += (y * z) * k[9] + (y * y * z) * k[16] + (y * z * z) * k[18];
    if constexpr (x * y * z != 0) p += (x * y * z) * k[19];
    return p;
}

// Hermite coefficients of f - f_eq from the raw ones of f (herm_acc on f):
// the equilibrium's are n (u u + (T - s) I) and n (u u u + (T - s)(u d)_sym),
// which the degree-7 quadrature integrates exactly.  dT = T - s (0 isothermal).
__device__ __forceinline__ void sub_eq_moments(double n, const double u[3], double dT, double a2[6], double a3[10])
{
    const double x = u[0], y = u[1], z = u[2];
    a2[0] -= n * (x * x + dT);
    a2[1] -= n * (y * y + dT);
    a2[2] -= n * (z * z + dT);
    a2[3] -= n * (x * y);
    a2[4] -= n * (x * z);
    a2[5] -= n * (y * z);
    a3[0] -= n * (x * x * x + 3.0 * dT * x);
    a3[1] -= n * (y * y * y + 3.0 * dT * y);
    a3[2] -= n * (z * z * z + 3.0 * dT * z);
    a3[3] -= n * (x * x * y + dT * y);
    a3[4] -= n * (x * x * z + dT * z);
    a3[5] -= n * (x * y * y + dT * x);
    a3[6] -= n * (y * y * z + dT * z);
    a3[7] -= n * (x * z * z + dT * x);
    a3[8] -= n * (y * z * z + dT * y);
    a3[9] -= n * (x * y * z);
}

// The post-collision value divided by w_i is a cubic polynomial in c_i:
//   n E(c) + (1 - 1/tau) P(c) + S(c),
// E the equilibrium (through h^(3); th1 = T/s - 1, 0 isothermal), P the
// projection (proj_coeffs), S the source (c.F/s; thermal: plus
// ((c.F)(c.u) - s F.u)/s^2 + Q (c^2 - 3 s)/(3 s^2)).  A[] holds its 20
// coefficients in the layout of proj_coeffs, evaluated per velocity by proj_of.
template <bool TH>
__device__ __forceinline__ void post_coeffs(double n, const double u[3], double th1, double om, const double F[3],
                                            double Q, const double a2[6], const double a3[10], double A[20])
{
    constexpr double is = 1.0 / CS2_39, is2 = is * is, is3 = is2 * is;
    const double x = u[0], y = u[1], z = u[2];
    proj_coeffs(a2, a3, A);
#pragma unroll
    for (int m = 0; m < 20; ++m) A[m] *= om;
    const double uu = (x * x + y * y + z * z) * is;
    const double g1 = (1.0 - 0.5 * uu - 2.5 * th1) * is;
    const double h2 = 0.5 * th1 * is, h3 = 0.5 * th1 * is2;
    A[0] += n * (1.0 - 0.5 * uu - 1.5 * th1);
    A[1] += n * (x * g1) + F[0] * is;
    A[2] += n * (y * g1) + F[1] * is;
    A[3] += n * (z * g1) + F[2] * is;
    A[4] += n * (0.5 * x * x * is2 + h2);
    A[5] += n * (0.5 * y * y * is2 + h2);
    A[6] += n * (0.5 * z * z * is2 + h2);
    A[7] += n * (x * y * is2);
    A[8] += n * (x * z * is2);
    A[9] += n * (y * z * is2);
    A[10] += n * (x * x * x * (is3 / 6.0) + h3 * x);
    A[11] += n * (y * y * y * (is3 / 6.0) + h3 * y);
    A[12] += n * (z * z * z * (is3 / 6.0) + h3 * z);
    A[13] += n * (0.5 * x * x * y * is3 + h3 * y);
    A[14] += n * (0.5 * x * x * z * is3 + h3 * z);
    A[15] += n * (0.5 * x * y * y * is3 + h3 * x);
    A[16] += n * (0.5 * y * y * z * is3 + h3 * z);
    A[17] += n * (0.5 * x * z * z * is3 + h3 * x);
    A[18] += n * (0.5 * y * z * z * is3 + h3 * y);
    A[19] += n * (x * y * z * is3);
    if constexpr (TH) {
        const double Fu = F[0] * x + F[1] * y + F[2] * z;
        A[0] -= (Fu + Q) * is;
        A[4] += (F[0] * x + Q * (1.0 / 3.0)) * is2;
        A[5] += (F[1] * y + Q * (1.0 / 3.0)) * is2;
        A[6] += (F[2] * z + Q * (1.0 / 3.0)) * is2;
        A[7] += (F[0] * y + F[1] * x) * is2;
        A[8] += (F[0] * z + F[2] * x) * is2;
        A[9] += (F[1] * z + F[2] * y) * is2;
    }
}

// Collide and stream of velocity I from node (x, y, z): post-collision value
// from the equilibrium, the relaxed projection and the first-order source,
// then the landing node.  A link that would leave the fluid layers is
// reversed at the wall plane: lateral run (2 d - |c_z|) c_a / |c_z| with d the
// node's distance to the plane, mirrored z.
// Thermal: the source adds the force's second Hermite order and the energy
// source on the trace of h^(2): w [((c.F)(c.u) - s F.u)/s^2 + Q (c^2 - 3 s)/(3 s^2)].
template <int I>
__device__ __forceinline__ void out39(const LatticeDev &L, double *__restrict__ fout, int x, int y, int z, double fp)
{
    constexpr int cx = C39X[I], cy = C39Y[I], cz = C39Z[I];
    int xt = x + cx, yt = y + cy, zt = z + cz, k = I;
    if constexpr (cz != 0) {
        if (L.zper) {
            zt = (zt < 0) ? zt + L.nz : ((zt >= L.nz) ? zt - L.nz : zt);
        } else {
            constexpr int az = cz < 0 ? -cz : cz;
            const int lo = L.wall_lo, hi = L.nz - L.wall_hi;
            int run = 0;
            bool hit = false;
            if constexpr (cz < 0) {
                if (zt < lo) {
                    run = 2 * (z - lo) + 1 + cz;
                    zt = 2 * lo - 1 - zt;
                    hit = true;
                }
            } else {
                if (zt >= hi) {
                    run = 2 * (hi - 1 - z) + 1 - cz;
                    zt = 2 * hi - 1 - zt;
                    hit = true;
                }
            }
            if (hit) {
                xt = x + (cx / az) * run;
                yt = y + (cy / az) * run;
                k = opp39(I);
            }
        }
    }
    xt = (xt < 0) ? xt + L.nx : ((xt >= L.nx) ? xt - L.nx : xt);
    yt = (yt < 0) ? yt + L.ny : ((yt >= L.ny) ? yt - L.ny : yt);
    __builtin_nontemporal_store(fp, fout + (size_t)k * L.pop_stride + (size_t)xt +
                                        (size_t)L.nx * ((size_t)yt + (size_t)L.ny * zt));
}

// The projections first (the populations are dead before the force's shell
// sum), the post-collision values and their streaming after it.
// Two forms of the same collision, chosen by measurement on the 64x64x136
// slit.  Isothermal: f - f_eq per velocity for the projection, and per velocity
// f_eq + (1 - 1/tau) w P(c) + w c.F/s (96 us; the polynomial form below took
// 100 us).  Thermal: the raw Hermite moments of f less the equilibrium's, and
// the whole post-collision value as one cubic polynomial per node (116 us
// against 159 us, at 228 VGPRs instead of ~320).
template <int... I>
__device__ __forceinline__ void project39(double n, const double u[3], const double *__restrict__ f, double a2[6],
                                          double a3[10], std::integer_sequence<int, I...>)
{
    const double uu_s = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / CS2_39;
    (herm_acc<I>(f[I] - feq39_of<I>(n, u, uu_s), a2, a3), ...);
}

template <int I>
__device__ __forceinline__ double post39(double fe, double om, const double K[20], const double F[3])
{
    const double cF = C39X[I] * F[0] + C39Y[I] * F[1] + C39Z[I] * F[2];
    return fe + om * (w39(I) * proj_of<I>(K)) + w39(I) * cF * (1.0 / CS2_39);
}

template <int... I>
__device__ __forceinline__ void emit39(const LatticeDev &L, double *__restrict__ fout, int x, int y, int z, double n,
                                      const double u[3], double om, const double F[3], const double a2[6],
                                      const double a3[10], std::integer_sequence<int, I...>)
{
    const double uu_s = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / CS2_39;
    double k[20];
    proj_coeffs(a2, a3, k);
    (out39<I>(L, fout, x, y, z, post39<I>(feq39_of<I>(n, u, uu_s), om, k, F)), ...);
}

template <int... I>
__device__ __forceinline__ void raw_herm39(const double *__restrict__ f, double a2[6], double a3[10],
                                           std::integer_sequence<int, I...>)
{
    (herm_acc<I>(f[I], a2, a3), ...);
}

template <int... I>
__device__ __forceinline__ void emit39_poly(const LatticeDev &L, double *__restrict__ fout, int x, int y, int z,
                                           const double A[20], std::integer_sequence<int, I...>)
{
    (out39<I>(L, fout, x, y, z, w39(I) * proj_of<I>(A)), ...);
}

// ------------------------------------------------- non-isothermal shell terms

// One element of the thermal shell sum, the lattice corner d of direction s
// (s scaled by 1/sqrt(2) on the face diagonals): with cur = s.(j' - n' u),
//   e1 = G [n' - chi kappa cur + n' (T' - T) / (2 T)]   (C^(1), along s)
//   e2 = G [-cur / 2 + n' (T' - T) / (sqrt(pi) v_T)]     (C^(2))
// Solid partners hold n' = j' = 0 and add nothing.
struct ThCtx {
    int x, y, zp;
    double u[3];
    double ckap;   // chi(z) * 2 / (v_T sqrt(pi))
    double T;      // T(r)
    double i2T;    // 1 / (2 T)
    double ipv;    // 1 / (sqrt(pi) v_T)
};

// LZ: z uniform over the block, the layer parts of the addresses scalar (as
// pair_element); otherwise one node index per read.
template <int DX, int DY, int DZ, int SX, int SY, int SZ, bool DIAG, bool LZ>
__device__ __forceinline__ void th_element(const Fields<double> &F, const LatticeDev &L, const ThCtx &c, double su,
                                           double &e1, double &e2)
{
    constexpr int SLOT = (DX & 1) | ((DY & 1) << 1) | ((DZ & 1) << 2);
    constexpr int BX = floordiv2(DX), BY = floordiv2(DY), BZ = floordiv2(DZ);
    double G, Tp, q[4];
    if constexpr (LZ) {
        const size_t lay = (size_t)L.plane;
        const char *njp = (const char *)F.nj + 32 * lay * (size_t)(c.zp + DZ);
        const char *tp = (const char *)F.T + 8 * lay * (size_t)(c.zp + DZ);
        const char *gz = (const char *)F.G + 8 * ((size_t)SLOT * L.fld_stride + lay * (size_t)(c.zp + BZ));
        G = *(const double *)(gz + (xb<BX, 8>(c.x, L.nx) + yb<BY, 8>(c.y, L.ny, L.nx)));
        Tp = *(const double *)(tp + (xb<DX, 8>(c.x, L.nx) + yb<DY, 8>(c.y, L.ny, L.nx)));
        load4((const double *)(njp + (xb<DX, 32>(c.x, L.nx) + yb<DY, 32>(c.y, L.ny, L.nx))), q);
    } else {
        const int ip = wrapc<DX>(c.x, L.nx) + L.nx * (wrapc<DY>(c.y, L.ny) + L.ny * (c.zp + DZ));
        const int gp = wrapc<BX>(c.x, L.nx) + L.nx * (wrapc<BY>(c.y, L.ny) + L.ny * (c.zp + BZ));
        G = F.G[SLOT * (size_t)L.fld_stride + gp];
        Tp = F.T[ip];
        load4(F.nj + 4 * (size_t)ip, q);
    }
    double sj = s_dot_j<SX, SY, SZ, double, double>(q);
    if constexpr (DIAG) sj *= 0.70710678118654752440;
    const double cur = sj - q[0] * su;
    const double ndT = q[0] * (Tp - c.T);
    e1 = G * (q[0] - c.ckap * cur + ndT * c.i2T);
    e2 = G * (-0.5 * cur + ndT * c.ipv);
}

template <int AX, int SG, int SIG, bool LZ>
__device__ __forceinline__ void th_axis(const Fields<double> &F, const LatticeDev &L, const ThCtx &c, double S[3],
                                        double &Qs)
{
    double e1, e2;
    th_element<AX == 0 ? SG * SIG : 0, AX == 1 ? SG * SIG : 0, AX == 2 ? SG * SIG : 0, AX == 0 ? SG : 0,
               AX == 1 ? SG : 0, AX == 2 ? SG : 0, false, LZ>(F, L, c, SG * c.u[AX], e1, e2);
    S[AX] += (1.0 / 30.0) * SG * e1;
    Qs += (1.0 / 30.0) * e2;
}

template <int PL, int SA, int SB, int LA, int LB, bool LZ>
__device__ __forceinline__ void th_corner(const Fields<double> &F, const LatticeDev &L, const ThCtx &c, double su,
                                          double al, double &d1, double &d2)
{
    using D = Diag<PL, SA, SB, LA, LB>;
    double e1, e2;
    th_element<D::DX, D::DY, D::DZ, D::SX, D::SY, D::SZ, true, LZ>(F, L, c, su, e1, e2);
    d1 += al * e1;
    d2 += al * e2;
}

template <int PL, int SA, int SB, int LL, bool LZ>
__device__ __forceinline__ void th_diag(const Fields<double> &F, const LatticeDev &L, const ThCtx &c,
                                        const double *alpha, double S[3], double &Qs)
{
    constexpr int A = (PL == 2) ? 1 : 0;
    constexpr int B = (PL == 0) ? 1 : 2;
    const double su = 0.70710678118654752440 * (SA * c.u[A] + SB * c.u[B]);
    double d1 = 0.0, d2 = 0.0;
    th_corner<PL, SA, SB, LL, LL, LZ>(F, L, c, su, alpha[0], d1, d2);
    th_corner<PL, SA, SB, LL, LL + 1, LZ>(F, L, c, su, alpha[1], d1, d2);
    th_corner<PL, SA, SB, LL + 1, LL, LZ>(F, L, c, su, alpha[2], d1, d2);
    th_corner<PL, SA, SB, LL + 1, LL + 1, LZ>(F, L, c, su, alpha[3], d1, d2);
    const double w = (1.0 / 15.0) * 0.70710678118654752440 * d1;
    S[A] += SA * w;
    S[B] += SB * w;
    Qs += (1.0 / 15.0) * d2;
}

template <int PL, int LL, bool LZ>
__device__ __forceinline__ void th_plane(const Fields<double> &F, const LatticeDev &L, const ThCtx &c,
                                         const double *alpha, double S[3], double &Qs)
{
    th_diag<PL, 1, 1, LL, LZ>(F, L, c, alpha, S, Qs);
    th_diag<PL, -1, -1, LL, LZ>(F, L, c, alpha, S, Qs);
    th_diag<PL, 1, -1, LL, LZ>(F, L, c, alpha, S, Qs);
    th_diag<PL, -1, 1, LL, LZ>(F, L, c, alpha, S, Qs);
}

// C^(1) with its temperature term, plus attraction and n g, and C^(2), at a
// fluid node with moments (n, u) and temperature T; v_T^2 = T.
template <int SIG, bool LZ>
__device__ __forceinline__ void th_node_force(const Fields<double> &F, const LatticeDev &L, const StepConst &sc,
                                              const double *__restrict__ chi, int x, int y, int z, double n,
                                              const double u[3], double T, double Fo[3], double &Qo)
{
    double S[3] = {0.0, 0.0, 0.0}, Qs = 0.0;
    const double vt = sqrt(T);
    if (sc.hs_on) {
        ThCtx c;
        c.x = x;
        c.y = y;
        c.zp = z + L.hz;
        c.u[0] = u[0];
        c.u[1] = u[1];
        c.u[2] = u[2];
        c.T = T;
        c.ckap = chi[z] * (2.0 / (vt * 1.7724538509055160273));
        c.i2T = 0.5 / T;
        c.ipv = 1.0 / (1.7724538509055160273 * vt);
        constexpr int LL = ell_of(SIG);
        th_axis<0, 1, SIG, LZ>(F, L, c, S, Qs);
        th_axis<0, -1, SIG, LZ>(F, L, c, S, Qs);
        th_axis<1, 1, SIG, LZ>(F, L, c, S, Qs);
        th_axis<1, -1, SIG, LZ>(F, L, c, S, Qs);
        th_axis<2, 1, SIG, LZ>(F, L, c, S, Qs);
        th_axis<2, -1, SIG, LZ>(F, L, c, S, Qs);
        th_plane<0, LL, LZ>(F, L, c, sc.alpha, S, Qs);
        th_plane<1, LL, LZ>(F, L, c, sc.alpha, S, Qs);
        th_plane<2, LL, LZ>(F, L, c, sc.alpha, S, Qs);
    }
    double Fa[3] = {0.0, 0.0, 0.0};
    if (sc.phi) att_force(L, sc, x, y, z, n, Fa);
    const double pn = -T * (double)(SIG * SIG) * 4.0 * M_PI * n;
    Fo[0] = pn * S[0] + Fa[0] + n * sc.g[0];
    Fo[1] = pn * S[1] + Fa[1] + n * sc.g[1];
    Fo[2] = pn * S[2] + Fa[2] + n * sc.g[2];
    Qo = -pn * Qs;
}

// Waves per SIMD the 39-velocity collide kernel is compiled for: the
// compiler's ~246 VGPRs allow 2; capping at 3 or 4 spills and measured 30 %
// and 100 % slower.
#ifndef HSLB_COLLIDE39_WAVES
#define HSLB_COLLIDE39_WAVES 2
#endif
#ifndef HSLB_COLLIDE39T_WAVES
#define HSLB_COLLIDE39T_WAVES 2
#endif

// 1-D grid over (fluid layer, chunk of 256 nodes of the layer), as k_collide.
template <int SIG, bool TH, int ROT = 0>
__global__ __launch_bounds__(256, TH ? HSLB_COLLIDE39T_WAVES : HSLB_COLLIDE39_WAVES) void k_collide39(LatticeDev L, StepConst sc, const double *__restrict__ chi,
                                                   const double *__restrict__ fin, double *__restrict__ fout,
                                                   Fields<double> fld, int cpp)
{
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int zl = lb / cpp;
    const int r = (lb - zl * cpp) * 256 + threadIdx.x;
    const int z = (L.zper ? 0 : L.wall_lo) + zl;
    if (r >= L.plane) return;
    const int y = r / L.nx;
    const int x = r - y * L.nx;
    const size_t id = (size_t)z * L.plane + r;
    // The populations stream through once per step and, at 39 x 8 bytes per
    // node, do not fit the last-level cache with the fields: non-temporal loads
    // and stores keep them from evicting the shell's moment fields
    // (95 against 110 us on the 64x64x136 slit).
    double f[Q39];
#pragma unroll
    for (int i = 0; i < Q39; ++i) f[i] = __builtin_nontemporal_load(fin + (size_t)i * L.pop_stride + id);
    double n = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q39; ++i) {
        n += f[i];
        jx += C39X[i] * f[i];
        jy += C39Y[i] * f[i];
        jz += C39Z[i] * f[i];
    }
    const double inv_n = (n != 0.0) ? 1.0 / n : 0.0;
    const double u[3] = {jx * inv_n, jy * inv_n, jz * inv_n};
    double T = 0.0;
    if constexpr (TH) {
        double e = 0.0;
#pragma unroll
        for (int i = 0; i < Q39; ++i) e += (double)(C39X[i] * C39X[i] + C39Y[i] * C39Y[i] + C39Z[i] * C39Z[i]) * f[i];
        T = (n != 0.0) ? (e * inv_n - (jx * jx + jy * jy + jz * jz) * inv_n * inv_n) / 3.0 : 0.0;
    }
    const double th1 = T / CS2_39 - 1.0;
    double a2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double a3[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double om = 1.0 - 1.0 / sc.tau;
    double Fv[3];
    if constexpr (TH) {
        raw_herm39(f, a2, a3, std::make_integer_sequence<int, Q39>{});
        sub_eq_moments(n, u, T - CS2_39, a2, a3);
        double Q;
        th_node_force<SIG, true>(fld, L, sc, chi, x, y, z, n, u, T, Fv, Q);
        double A[20];
        post_coeffs<true>(n, u, th1, om, Fv, Q, a2, a3, A);
        emit39_poly(L, fout, x, y, z, A, std::make_integer_sequence<int, Q39>{});
    } else {
        project39(n, u, f, a2, a3, std::make_integer_sequence<int, Q39>{});
        node_force<SIG, true, double, false, false, ROT>(fld, L, sc, chi, x, y, z, n, u, Fv);
        emit39(L, fout, x, y, z, n, u, om, Fv, a2, a3, std::make_integer_sequence<int, Q39>{});
    }
}

template <int SIG, bool TH>
__global__ __launch_bounds__(256) void k_force39(LatticeDev L, StepConst sc, const double *__restrict__ chi,
                                                 const double *__restrict__ f, Fields<double> fld,
                                                 double *__restrict__ Fout, double *__restrict__ Qout)
{
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= L.N) return;
    const int z = id / L.plane;
    const int rem = id - z * L.plane;
    const int y = rem / L.nx;
    const int x = rem - y * L.nx;
    double Fv[3] = {0.0, 0.0, 0.0}, Q = 0.0;
    if (is_fluid_z(L, z)) {
        double n, jx, jy, jz, e;
        moments39e(L, f, id, z, n, jx, jy, jz, e);
        const double inv_n = (n != 0.0) ? 1.0 / n : 0.0;
        const double u[3] = {jx * inv_n, jy * inv_n, jz * inv_n};
        if constexpr (TH)
            th_node_force<SIG, false>(fld, L, sc, chi, x, y, z, n, u, temp_of(n, jx, jy, jz, e), Fv, Q);
        else
            node_force<SIG, false, double, false>(fld, L, sc, chi, x, y, z, n, u, Fv);
    }
    Fout[id] = Fv[0];
    Fout[L.N + id] = Fv[1];
    Fout[2 * (size_t)L.N + id] = Fv[2];
    if (Qout) Qout[id] = Q;
}

inline unsigned blocks_for(int n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename TM>
hipError_t launch_attraction(hipStream_t s, const LatticeDev &L, const AttWeights &aw, const TM *n, double *a,
                             double *b, double *phi)
{
    if (aw.R < 0 || aw.R > ATT_MAX_R) return hipErrorInvalidValue;
    const dim3 g(blocks_for(L.plane), L.nz), blk(256);
    if (L.nx == 64)  // a wave per x-row: the taps from the neighbouring lanes
        hipLaunchKernelGGL((k_att_x<TM, 1>), g, blk, 0, s, L, aw, n, a);
    else if (L.nx == 16)
        hipLaunchKernelGGL((k_att_x<TM, 2>), g, blk, 0, s, L, aw, n, a);
    else
        hipLaunchKernelGGL((k_att_x<TM>), g, blk, 0, s, L, aw, n, a);
    hipLaunchKernelGGL(k_att_y, g, blk, 0, s, L, aw, a, b);
    hipLaunchKernelGGL(k_att_z, g, blk, 0, s, L, aw, b, phi);
    return hipGetLastError();
}

hipError_t launch_round_f32(hipStream_t s, double *a, int count)
{
    hipLaunchKernelGGL(k_round_f32, dim3(blocks_for(count)), dim3(256), 0, s, a, count);
    return hipGetLastError();
}

hipError_t launch_feq39(hipStream_t s, const LatticeDev &L, const double *n, const double *u, const double *T,
                        double *out)
{
    hipLaunchKernelGGL(k_feq39, dim3(blocks_for(L.N)), dim3(256), 0, s, L, n, u, T, out);
    return hipGetLastError();
}

hipError_t launch_moments39(hipStream_t s, const LatticeDev &L, const double *f, Fields<double> fld, bool thermal)
{
    if (thermal && !fld.T) return hipErrorInvalidValue;
    const dim3 g(blocks_for(L.plane), L.nz), b(256);
    if (thermal)
        hipLaunchKernelGGL(k_moments39<true>, g, b, 0, s, L, f, fld);
    else
        hipLaunchKernelGGL(k_moments39<false>, g, b, 0, s, L, f, fld);
    return hipGetLastError();
}

hipError_t launch_moments39_rs(hipStream_t s, const LatticeDev &L, int sigma, const double *f, Fields<double> fld,
                               bool thermal, double *rs)
{
    if (256 % L.nx != 0 || L.plane % 256 != 0) return hipErrorInvalidValue;
    if (thermal && !fld.T) return hipErrorInvalidValue;
    const dim3 g(L.plane / 256, L.nz), b(256);
#define HSLB_M39(SG)                                                                               \
    case SG:                                                                                       \
        if (thermal)                                                                               \
            hipLaunchKernelGGL((k_moments39_rs<SG, true>), g, b, 0, s, L, f, fld, rs);             \
        else                                                                                       \
            hipLaunchKernelGGL((k_moments39_rs<SG, false>), g, b, 0, s, L, f, fld, rs);            \
        break;
    switch (sigma) {
        HSLB_M39(2)
        HSLB_M39(3)
        HSLB_M39(4)
        HSLB_M39(5)
        HSLB_M39(6)
        HSLB_M39(7)
        HSLB_M39(8)
    default: return hipErrorInvalidValue;
    }
#undef HSLB_M39
    return hipGetLastError();
}

hipError_t launch_profiles39(hipStream_t s, const LatticeDev &L, const double *f, double *out)
{
    hipLaunchKernelGGL(k_profiles39, dim3(L.nz), dim3(256), 0, s, L, f, out);
    return hipGetLastError();
}

hipError_t launch_export39(hipStream_t s, const LatticeDev &L, const double *f, double *n, double *u)
{
    hipLaunchKernelGGL(k_export39, dim3(blocks_for(L.N)), dim3(256), 0, s, L, f, n, u);
    return hipGetLastError();
}

hipError_t launch_collide39(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c, const double *chi,
                            const double *fin, double *fout, Fields<double> fld, bool thermal)
{
    if (thermal && !fld.T) return hipErrorInvalidValue;
    const int layers = L.zper ? L.nz : L.nz - L.wall_lo - L.wall_hi;
    const int cpp = (int)blocks_for(L.plane);
    const dim3 g(cpp * layers), b(256);
    // a wave per x-row of 64 nodes: x-neighbour (n, j) reads shared between lanes
    const bool rot = L.nx == 64;
#define HSLB_C39(SG)                                                                                  \
    case SG:                                                                                          \
        if (thermal)                                                                                  \
            hipLaunchKernelGGL((k_collide39<SG, true>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp);    \
        else if (rot)                                                                                 \
            hipLaunchKernelGGL((k_collide39<SG, false, 1>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp); \
        else                                                                                          \
            hipLaunchKernelGGL((k_collide39<SG, false>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp);   \
        break;
    switch (sigma) {
        HSLB_C39(2)
        HSLB_C39(3)
        HSLB_C39(4)
        HSLB_C39(5)
        HSLB_C39(6)
        HSLB_C39(7)
        HSLB_C39(8)
    default: return hipErrorInvalidValue;
    }
#undef HSLB_C39
    return hipGetLastError();
}

hipError_t launch_force39(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c, const double *chi,
                          const double *f, Fields<double> fld, bool thermal, double *F, double *Q)
{
    if (thermal && !fld.T) return hipErrorInvalidValue;
    const dim3 g(blocks_for(L.N)), b(256);
#define HSLB_F39(SG)                                                                               \
    case SG:                                                                                       \
        if (thermal)                                                                               \
            hipLaunchKernelGGL((k_force39<SG, true>), g, b, 0, s, L, c, chi, f, fld, F, Q);          \
        else                                                                                       \
            hipLaunchKernelGGL((k_force39<SG, false>), g, b, 0, s, L, c, chi, f, fld, F, Q);         \
        break;
    switch (sigma) {
        HSLB_F39(2)
        HSLB_F39(3)
        HSLB_F39(4)
        HSLB_F39(5)
        HSLB_F39(6)
        HSLB_F39(7)
        HSLB_F39(8)
    default: return hipErrorInvalidValue;
    }
#undef HSLB_F39
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, const void *src, void *dst, size_t bytes)
{
    const size_t n = bytes / 16;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const float4 *)src, (float4 *)dst, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers

hipError_t launch_feq(hipStream_t s, const LatticeDev &L, const double *n, const double *u, double *out)
{
    hipLaunchKernelGGL(k_feq, dim3(blocks_for(L.N)), dim3(256), 0, s, L, n, u, out);
    return hipGetLastError();
}

template <typename TF>
hipError_t launch_layer_means(hipStream_t s, const LatticeDev &L, const TF *f, int stride, const double *ref,
                              double *out)
{
    hipLaunchKernelGGL(k_layer_means<TF>, dim3(L.nz), dim3(256), 0, s, L, f, stride, ref, out);
    return hipGetLastError();
}

template <typename TF, typename TM>
hipError_t launch_moments(hipStream_t s, const LatticeDev &L, const double *nref, const TF *f, Fields<TM> fld)
{
    hipLaunchKernelGGL((k_moments<TF, TM>), dim3(blocks_for(L.plane), L.nz), dim3(256), 0, s, L, nref, f, fld);
    return hipGetLastError();
}

template <typename TM>
hipError_t launch_smooth2(hipStream_t s, const LatticeDev &L, int sigma, double eta_pref, Fields<TM> fld,
                          TM *rs)
{
    const dim3 b(256);
    const int R = sigma / 2;
    const dim3 g1(blocks_for(L.plane), L.nz + 2 * R), g2(blocks_for(L.plane), L.nz);
#define HSLB_S2(SG)                                                                                \
    case SG:                                                                                       \
        hipLaunchKernelGGL((k_rowsum<SG, TM>), g1, b, 0, s, L, fld, rs);                           \
        hipLaunchKernelGGL((k_ballsum<SG, TM>), g2, b, 0, s, L, eta_pref, fld, (const TM *)rs);    \
        break;
    switch (sigma) {
        HSLB_S2(2)
        HSLB_S2(3)
        HSLB_S2(4)
        HSLB_S2(5)
        HSLB_S2(6)
        HSLB_S2(7)
        HSLB_S2(8)
    default: return hipErrorInvalidValue;
    }
#undef HSLB_S2
    return hipGetLastError();
}

template <typename TF, typename TM>
hipError_t launch_moments_rs(hipStream_t s, const LatticeDev &L, int sigma, const double *nref, const TF *f,
                             Fields<TM> fld, TM *rs, bool write_n)
{
    if (256 % L.nx != 0 || L.plane % 256 != 0) return hipErrorInvalidValue;
    const dim3 g(L.plane / 256, L.nz), b(256);
    // (n, j) and the row sums beyond the 256 MiB last-level cache are stored
    // non-temporally, as the contact values are (256^3 bulk: 282 MB each)
    const int nt = 4.0 * sizeof(TM) * (double)L.fld_stride > HSLB_NT_FIELD_MIB * 1024.0 * 1024.0 ? 1 : 0;
    switch (sigma) {
    case 2: hipLaunchKernelGGL((k_moments_rs<2, TF, TM>), g, b, 0, s, L, nref, f, fld, rs, (int)write_n, nt); break;
    case 3: hipLaunchKernelGGL((k_moments_rs<3, TF, TM>), g, b, 0, s, L, nref, f, fld, rs, (int)write_n, nt); break;
    case 4: hipLaunchKernelGGL((k_moments_rs<4, TF, TM>), g, b, 0, s, L, nref, f, fld, rs, (int)write_n, nt); break;
    case 5: hipLaunchKernelGGL((k_moments_rs<5, TF, TM>), g, b, 0, s, L, nref, f, fld, rs, (int)write_n, nt); break;
    case 6: hipLaunchKernelGGL((k_moments_rs<6, TF, TM>), g, b, 0, s, L, nref, f, fld, rs, (int)write_n, nt); break;
    case 7: hipLaunchKernelGGL((k_moments_rs<7, TF, TM>), g, b, 0, s, L, nref, f, fld, rs, (int)write_n, nt); break;
    case 8: hipLaunchKernelGGL((k_moments_rs<8, TF, TM>), g, b, 0, s, L, nref, f, fld, rs, (int)write_n, nt); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TM>
hipError_t launch_ballsum(hipStream_t s, const LatticeDev &L, int sigma, double eta_pref, Fields<TM> fld, const TM *rs)
{
    const dim3 g(blocks_for(L.plane), L.nz), b(256);
    switch (sigma) {
    case 2: hipLaunchKernelGGL((k_ballsum<2, TM>), g, b, 0, s, L, eta_pref, fld, rs); break;
    case 3: hipLaunchKernelGGL((k_ballsum<3, TM>), g, b, 0, s, L, eta_pref, fld, rs); break;
    case 4: hipLaunchKernelGGL((k_ballsum<4, TM>), g, b, 0, s, L, eta_pref, fld, rs); break;
    case 5: hipLaunchKernelGGL((k_ballsum<5, TM>), g, b, 0, s, L, eta_pref, fld, rs); break;
    case 6: hipLaunchKernelGGL((k_ballsum<6, TM>), g, b, 0, s, L, eta_pref, fld, rs); break;
    case 7: hipLaunchKernelGGL((k_ballsum<7, TM>), g, b, 0, s, L, eta_pref, fld, rs); break;
    case 8: hipLaunchKernelGGL((k_ballsum<8, TM>), g, b, 0, s, L, eta_pref, fld, rs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TM>
hipError_t launch_gfield(hipStream_t s, const LatticeDev &L, int g2_model, Fields<TM> fld)
{
    const double g_bytes = 7.0 * (double)L.fld_stride * sizeof(TM);
    const dim3 g(blocks_for(L.plane), L.nz);
    if (g_bytes > HSLB_NT_FIELD_MIB * 1024.0 * 1024.0)
        hipLaunchKernelGGL((k_gfield<TM, true>), g, dim3(256), 0, s, L, g2_model, fld);
    else if (L.nx == 64)  // a wave per x-row: the x + 1 values from the neighbouring lane
        hipLaunchKernelGGL((k_gfield<TM, false, 1>), g, dim3(256), 0, s, L, g2_model, fld);
    else if (L.nx == 16)  // a 16-lane row per x-row
        hipLaunchKernelGGL((k_gfield<TM, false, 2>), g, dim3(256), 0, s, L, g2_model, fld);
    else
        hipLaunchKernelGGL((k_gfield<TM, false>), g, dim3(256), 0, s, L, g2_model, fld);
    return hipGetLastError();
}

template <typename TF, typename TM, bool M, bool NT, int ROT = 0>
hipError_t launch_collide_t(hipStream_t s, int sigma, dim3 g, dim3 b, const LatticeDev &L, const StepConst &c,
                            const double *chi, const TF *fin, TF *fout, Fields<TM> fld, int cpp, int band);

bool collide_tiles_apply(const LatticeDev &L, int sigma, const StepConst &c, bool fp32)
{
    return fp32 && !c.links && c.hs_on && sigma >= 2 && sigma <= 8 && L.nx % stage::TX == 0 &&
           L.ny % stage::TY == 0;
}

template <bool NT>
hipError_t launch_collide_tiles_t(hipStream_t s, int sigma, int layers, const LatticeDev &L, const StepConst &c,
                                  const double *chi, const float *fin, float *fout, Fields<float> fld)
{
    const dim3 g((unsigned)(layers * (L.nx / stage::TX) * (L.ny / stage::TY))), b(256);
    switch (sigma) {
    case 2: hipLaunchKernelGGL((k_collide_tiles<2, NT>), g, b, 0, s, L, c, chi, fin, fout, fld); break;
    case 3: hipLaunchKernelGGL((k_collide_tiles<3, NT>), g, b, 0, s, L, c, chi, fin, fout, fld); break;
    case 4: hipLaunchKernelGGL((k_collide_tiles<4, NT>), g, b, 0, s, L, c, chi, fin, fout, fld); break;
    case 5: hipLaunchKernelGGL((k_collide_tiles<5, NT>), g, b, 0, s, L, c, chi, fin, fout, fld); break;
    case 6: hipLaunchKernelGGL((k_collide_tiles<6, NT>), g, b, 0, s, L, c, chi, fin, fout, fld); break;
    case 7: hipLaunchKernelGGL((k_collide_tiles<7, NT>), g, b, 0, s, L, c, chi, fin, fout, fld); break;
    case 8: hipLaunchKernelGGL((k_collide_tiles<8, NT>), g, b, 0, s, L, c, chi, fin, fout, fld); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_collide_tiles(hipStream_t s, int sigma, int layers, bool nt, const LatticeDev &L,
                                const StepConst &c, const double *chi, const float *fin, float *fout,
                                Fields<float> fld)
{
    return nt ? launch_collide_tiles_t<true>(s, sigma, layers, L, c, chi, fin, fout, fld)
              : launch_collide_tiles_t<false>(s, sigma, layers, L, c, chi, fin, fout, fld);
}


template <typename TF, typename TM>
hipError_t launch_collide(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c, const double *chi,
                          const TF *fin, TF *fout, Fields<TM> fld, bool tiles)
{
    const int layers = L.zper ? L.nz : L.nz - L.wall_lo - L.wall_hi;
    const int cpp = (int)blocks_for(L.plane);
    const dim3 g(cpp * layers), b(256);
    // Bands of the layer per XCD once a band spans at least two shell
    // diameters in y: 256^3 bulk (sigma 6, 32-row bands) 1486 -> 1399 us,
    // 128 x 128 slit (sigma 8, 16 rows) 338 -> 320 us; the 64 x 64 slit
    // (sigma 8, 8-row bands) keeps z slabs, 39.6 against 41.9 us.  Splitting
    // each band's layers over 2 or 4 XCDs (wider bands) measured in between.
    const int band = (cpp % 8 == 0 && L.ny >= 16 * sigma) ? 1 : 0;
    if (c.links) return launch_collide_t<TF, TM, true, false>(s, sigma, g, b, L, c, chi, fin, fout, fld, cpp, band);
    // populations beyond the last-level cache (two copies over 128 MiB) stream
    // non-temporally
    const double pop_bytes = 2.0 * NQ * (double)L.pop_stride * sizeof(TF);
    if constexpr (std::is_same<TF, float>::value && std::is_same<TM, float>::value) {
        if (tiles && collide_tiles_apply(L, sigma, c, true))
            return launch_collide_tiles(s, sigma, layers, pop_bytes > 128.0 * 1024 * 1024, L, c, chi, fin, fout, fld);
    }
    if (pop_bytes > 128.0 * 1024 * 1024) {
        // x-rows of 128 or 256 nodes over 2 or 4 waves: lanes share x-neighbour
        // reads, the row-edge lanes through the block's LDS (256^3 bulk 1401 ->
        // 1373 us; the cache-resident 128 x 128 slit lost, 315 -> 366 us, so
        // only this instance takes it)
        if constexpr (std::is_same<TF, float>::value && std::is_same<TM, float>::value) {
            if ((L.nx == 128 || L.nx == 256) && L.plane % 256 == 0 && sigma >= 2)
                return launch_collide_t<TF, TM, false, true, 3>(s, sigma, g, b, L, c, chi, fin, fout, fld, cpp, band);
        }
        return launch_collide_t<TF, TM, false, true>(s, sigma, g, b, L, c, chi, fin, fout, fld, cpp, band);
    }
    // a wave per x-row of 64 nodes: x-neighbour (n, j) reads shared between
    // lanes (benchmark slit 39.9 -> 36.7 us)
    if constexpr (std::is_same<TF, float>::value && std::is_same<TM, float>::value) {
        if (L.nx == 64)
            return launch_collide_t<TF, TM, false, false, 1>(s, sigma, g, b, L, c, chi, fin, fout, fld, cpp, band);
    }
    return launch_collide_t<TF, TM, false, false>(s, sigma, g, b, L, c, chi, fin, fout, fld, cpp, band);
}

template <typename TF, typename TM, bool M, bool NT, int ROT>
hipError_t launch_collide_t(hipStream_t s, int sigma, dim3 g, dim3 b, const LatticeDev &L, const StepConst &c,
                            const double *chi, const TF *fin, TF *fout, Fields<TM> fld, int cpp, int band)
{
    switch (sigma) {
    case 0: hipLaunchKernelGGL((k_collide<0, TF, TM, M, NT, ROT>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp, band); break;
    case 2: hipLaunchKernelGGL((k_collide<2, TF, TM, M, NT, ROT>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp, band); break;
    case 3: hipLaunchKernelGGL((k_collide<3, TF, TM, M, NT, ROT>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp, band); break;
    case 4: hipLaunchKernelGGL((k_collide<4, TF, TM, M, NT, ROT>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp, band); break;
    case 5: hipLaunchKernelGGL((k_collide<5, TF, TM, M, NT, ROT>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp, band); break;
    case 6: hipLaunchKernelGGL((k_collide<6, TF, TM, M, NT, ROT>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp, band); break;
    case 7: hipLaunchKernelGGL((k_collide<7, TF, TM, M, NT, ROT>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp, band); break;
    case 8: hipLaunchKernelGGL((k_collide<8, TF, TM, M, NT, ROT>), g, b, 0, s, L, c, chi, fin, fout, fld, cpp, band); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TF, typename TM>
hipError_t launch_force(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c, const double *chi,
                        const TF *f, Fields<TM> fld, double *F)
{
    const dim3 g(blocks_for(L.N)), b(256);
    switch (sigma) {
    case 2: hipLaunchKernelGGL((k_force<2, TF, TM>), g, b, 0, s, L, c, chi, f, fld, F); break;
    case 3: hipLaunchKernelGGL((k_force<3, TF, TM>), g, b, 0, s, L, c, chi, f, fld, F); break;
    case 4: hipLaunchKernelGGL((k_force<4, TF, TM>), g, b, 0, s, L, c, chi, f, fld, F); break;
    case 5: hipLaunchKernelGGL((k_force<5, TF, TM>), g, b, 0, s, L, c, chi, f, fld, F); break;
    case 6: hipLaunchKernelGGL((k_force<6, TF, TM>), g, b, 0, s, L, c, chi, f, fld, F); break;
    case 7: hipLaunchKernelGGL((k_force<7, TF, TM>), g, b, 0, s, L, c, chi, f, fld, F); break;
    case 8: hipLaunchKernelGGL((k_force<8, TF, TM>), g, b, 0, s, L, c, chi, f, fld, F); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TF>
hipError_t launch_profiles_pop(hipStream_t s, const LatticeDev &L, const double *nref, const TF *f, double *out)
{
    hipLaunchKernelGGL(k_profiles<TF>, dim3(L.nz), dim3(256), 0, s, L, nref, f, out);
    return hipGetLastError();
}

template <typename TM>
hipError_t launch_unpad(hipStream_t s, const LatticeDev &L, const TM *src, double *dst)
{
    hipLaunchKernelGGL(k_unpad<TM>, dim3(blocks_for(L.N)), dim3(256), 0, s, L, src, dst);
    return hipGetLastError();
}

template <typename TF>
hipError_t launch_export_moments(hipStream_t s, const LatticeDev &L, const double *nref, const TF *f, double *n,
                                 double *u)
{
    hipLaunchKernelGGL(k_export_moments<TF>, dim3(blocks_for(L.N)), dim3(256), 0, s, L, nref, f, n, u);
    return hipGetLastError();
}

template <typename TF>
hipError_t launch_get_pop(hipStream_t s, const LatticeDev &L, const double *nref, const TF *f, double *out)
{
    hipLaunchKernelGGL(k_get_pop<TF>, dim3(blocks_for(L.N)), dim3(256), 0, s, L, nref, f, out);
    return hipGetLastError();
}

template <typename TF>
hipError_t launch_set_pop(hipStream_t s, const LatticeDev &L, const double *nref, const double *in, TF *f)
{
    hipLaunchKernelGGL(k_set_pop<TF>, dim3(blocks_for(L.N)), dim3(256), 0, s, L, nref, in, f);
    return hipGetLastError();
}

template <typename TF>
hipError_t launch_batch_layer_means(hipStream_t s, const SlitDesc *desc, const WorkItem *items, int nitems,
                                    const TF *f)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_layer_means<TF>, dim3(nitems), dim3(256), 0, s, desc, items, f);
    return hipGetLastError();
}

template <typename TF, typename TM>
hipError_t launch_batch_phase(hipStream_t s, int phase, unsigned grid, const SlitDesc *desc, const WorkItem *work,
                              int nwork, const TF *fin, TF *fout, Fields<TM> fld, TM *rs, const double *chi,
                              bool rows16)
{
    if (nwork <= 0) return hipSuccess;
    if (rows16 && phase == 3)
        hipLaunchKernelGGL((kb_phase<TF, TM, 2>), dim3(grid), dim3(256), 0, s, phase, desc, work, nwork, fin, fout,
                           fld, rs, chi);
    else
        hipLaunchKernelGGL((kb_phase<TF, TM>), dim3(grid), dim3(256), 0, s, phase, desc, work, nwork, fin, fout, fld,
                           rs, chi);
    return hipGetLastError();
}

template <typename TF, typename TM>
hipError_t launch_batch_collide(hipStream_t s, unsigned grid, const SlitDesc *desc, const WorkItem *work, int nwork,
                                const TF *fin, TF *fout, Fields<TM> fld, const double *chi, bool rows16)
{
    if (nwork <= 0) return hipSuccess;
    if constexpr (std::is_same<TF, float>::value && std::is_same<TM, float>::value) {
        if (rows16) {
            hipLaunchKernelGGL((kb_collide<TF, TM, 2>), dim3(grid), dim3(256), 0, s, desc, work, nwork, fin, fout,
                               fld, chi);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((kb_collide<TF, TM, 0>), dim3(grid), dim3(256), 0, s, desc, work, nwork, fin, fout, fld, chi);
    return hipGetLastError();
}

template <typename TF>
hipError_t launch_batch_profiles(hipStream_t s, const SlitDesc *desc, const WorkItem *items, int nitems,
                                 const int *prof_off, const TF *f, double *out)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_profiles<TF>, dim3(nitems), dim3(256), 0, s, desc, items, prof_off, f, out);
    return hipGetLastError();
}

#define HSLB_INST_TF(TF)                                                                                  \
    template hipError_t launch_layer_means<TF>(hipStream_t, const LatticeDev &, const TF *, int,          \
                                               const double *, double *);                                 \
    template hipError_t launch_batch_layer_means<TF>(hipStream_t, const SlitDesc *, const WorkItem *, int, \
                                                     const TF *);                                         \
    template hipError_t launch_profiles_pop<TF>(hipStream_t, const LatticeDev &, const double *,          \
                                                const TF *, double *);                                    \
    template hipError_t launch_get_pop<TF>(hipStream_t, const LatticeDev &, const double *, const TF *,   \
                                           double *);                                                     \
    template hipError_t launch_export_moments<TF>(hipStream_t, const LatticeDev &, const double *,        \
                                                  const TF *, double *, double *);                        \
    template hipError_t launch_set_pop<TF>(hipStream_t, const LatticeDev &, const double *,               \
                                           const double *, TF *);                                         \
    template hipError_t launch_batch_profiles<TF>(hipStream_t, const SlitDesc *, const WorkItem *, int,     \
                                                  const int *, const TF *, double *);
#define HSLB_INST_TM(TM)                                                                              \
    template hipError_t launch_gfield<TM>(hipStream_t, const LatticeDev &, int, Fields<TM>);         \
    template hipError_t launch_attraction<TM>(hipStream_t, const LatticeDev &, const AttWeights &,   \
                                              const TM *, double *, double *, double *);             \
    template hipError_t launch_smooth2<TM>(hipStream_t, const LatticeDev &, int, double, Fields<TM>, TM *); \
    template hipError_t launch_ballsum<TM>(hipStream_t, const LatticeDev &, int, double, Fields<TM>, const TM *); \
    template hipError_t launch_unpad<TM>(hipStream_t, const LatticeDev &, const TM *, double *);
#define HSLB_INST_TFTM(TF, TM)                                                                              \
    template hipError_t launch_moments<TF, TM>(hipStream_t, const LatticeDev &, const double *, const TF *, \
                                               Fields<TM>);                                                 \
    template hipError_t launch_moments_rs<TF, TM>(hipStream_t, const LatticeDev &, int, const double *,      \
                                                  const TF *, Fields<TM>, TM *, bool);                      \
    template hipError_t launch_collide<TF, TM>(hipStream_t, const LatticeDev &, int, const StepConst &,    \
                                               const double *, const TF *, TF *, Fields<TM>, bool);         \
    template hipError_t launch_force<TF, TM>(hipStream_t, const LatticeDev &, int, const StepConst &,      \
                                             const double *, const TF *, Fields<TM>, double *);              \
    template hipError_t launch_batch_phase<TF, TM>(hipStream_t, int, unsigned, const SlitDesc *,            \
                                                   const WorkItem *, int, const TF *, TF *, Fields<TM>, TM *, \
                                                   const double *, bool);                                          \
    template hipError_t launch_batch_collide<TF, TM>(hipStream_t, unsigned, const SlitDesc *,               \
                                                     const WorkItem *, int, const TF *, TF *, Fields<TM>,     \
                                                     const double *, bool);

// ------------------------------------------------ allocation-free scratch

namespace {

// The scratch of hslb_force_noalloc.  Host code reaches it only through the
// address scratch_address looked up for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

__global__ __launch_bounds__(256) void k_fill(double *__restrict__ a, size_t count, double v)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) a[i] = v;
}

__global__ __launch_bounds__(256) void k_chi(LatticeDev L, int sigma, int wall_reg, double *__restrict__ chi)
{
    const int z = blockIdx.x * 256 + threadIdx.x;
    if (z >= L.nz) return;
    double c = 1.0;
    if (!L.zper && wall_reg) {
        const double za = L.wall_lo - 0.5, zb = L.nz - L.wall_hi - 0.5;
        c = 1.0 - exp(-fmin((double)z - za, zb - (double)z) / (double)sigma);
    }
    chi[z] = c;
}

}  // namespace

hipError_t scratch_address(void **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_fill(hipStream_t s, double *a, size_t count, double v)
{
    if (count == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, a, count, v);
    return hipGetLastError();
}

hipError_t launch_chi(hipStream_t s, const LatticeDev &L, int sigma, int wall_reg, double *chi)
{
    hipLaunchKernelGGL(k_chi, dim3((L.nz + 255) / 256), dim3(256), 0, s, L, sigma, wall_reg, chi);
    return hipGetLastError();
}

HSLB_INST_TF(float)
HSLB_INST_TF(double)
HSLB_INST_TM(float)
HSLB_INST_TM(double)
HSLB_INST_TFTM(float, float)
HSLB_INST_TFTM(double, double)

}  // namespace hslb
