// Internal declarations shared by the host engine and the HIP kernels of
// libhslb.so.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hslb {

constexpr int NQ = 19;
// D3Q19 velocities and opposite directions (host and device)
constexpr int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[NQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// The 39-velocity third-order lattice in the public population order: rest,
// axis length 1, cube diagonals, axis length 2, (2, 2, 0) family, axis
// length 3; every odd index is followed by its opposite.
constexpr int Q39 = 39;
constexpr int C39X[Q39] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1, 2, -2, 0, 0, 0,
                           0, 2, -2, 2, -2, 2, -2, 2, -2, 0, 0, 0, 0, 3, -3, 0, 0, 0, 0};
constexpr int C39Y[Q39] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 0, 0, 2, -2, 0,
                           0, 2, -2, -2, 2, 0, 0, 0, 0, 2, -2, 2, -2, 0, 0, 3, -3, 0, 0};
constexpr int C39Z[Q39] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0, 2,
                           -2, 0, 0, 0, 0, 2, -2, -2, 2, 2, -2, -2, 2, 0, 0, 0, 0, 3, -3};
__host__ __device__ constexpr int opp39(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// Weight by |c|^2: 0 and 1 -> 1/12, 3 -> 1/27, 4 -> 2/135, 8 -> 1/432, 9 -> 1/1620.
__host__ __device__ constexpr double w39(int i)
{
    const int c2 = C39X[i] * C39X[i] + C39Y[i] * C39Y[i] + C39Z[i] * C39Z[i];
    return c2 <= 1 ? 1.0 / 12.0 : c2 == 3 ? 1.0 / 27.0 : c2 == 4 ? 2.0 / 135.0 : c2 == 8 ? 1.0 / 432.0 : 1.0 / 1620.0;
}
constexpr double CS2_39 = 2.0 / 3.0;  // v_T^2 of the 39-velocity lattice

constexpr int NGSLOT = 7;  // contact-value sub-lattices: bits x=1, y=2, z=4 (0..6)

// Workgroups are handed to the 8 XCDs round-robin by linear block index.  This
// bijection of [0, nb) gives XCD x a contiguous run of logical blocks, so that
// a stencil's neighbouring planes stay in that XCD's L2 instead of being
// fetched by all eight.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int q = nb >> 3, rm = nb & 7;
    const int x = b & 7, slot = b >> 3;
    return x * q + (x < rm ? x : rm) + slot;
}

// The other bijection for a grid of (layer, chunk) blocks, layers * cpp of
// them with cpp (chunks per layer) a multiple of 8, b the linear block index
// (a 2-D grid (cpp, layers) passes blockIdx.x + cpp * blockIdx.y): XCD x takes chunks
// [x cpp/8, (x+1) cpp/8) of every layer, layer by layer, so that all XCDs move
// through z together and each keeps a narrow band of the layers in its L2.
// Returns the block's layer zl and chunk c.
__device__ __forceinline__ void xcd_band(int b, int cpp, int &zl, int &c)
{
    const int x = b & 7, slot = b >> 3, bw = cpp >> 3;
    zl = slot / bw;
    c = x * bw + (slot - zl * bw);
}

// Geometry of one lattice as the kernels see it.
//  - populations: [19][pop_stride], node = x + nx*(y + ny*z), z in [0, nz)
//  - padded fields (n, j, eta_bar, G): [.. ][fld_stride] with hz ghost/zero
//    layers below and above: index = x + nx*(y + ny*(z + hz))
struct LatticeDev {
    int nx, ny, nz;
    int wall_lo, wall_hi;
    int zper;        // 1: z periodic (no walls)
    int hz;          // z halo of the padded fields
    int plane;       // nx*ny
    int N;           // nx*ny*nz
    int pop_stride;  // >= N
    int fld_stride;  // >= nx*ny*(nz + 2 hz)
};

// Per-step constants (uniform across the grid).
struct StepConst {
    double tau;
    double g[3];        // external force per particle
    // Populations are stored as f_i - ref[z][i], ref[z] the layer means of the
    // 19 populations ([nz][19] doubles); the collide kernel reads with nref_r
    // and writes with nref_w (equal except on a refresh step).
    const double *nref_r;
    const double *nref_w;
    double pref;        // -v_T^2 sigma^2 4 pi
    double kappa;       // 2 / (v_T sqrt(pi))
    double eta_pref;    // (pi sigma^3 / 6) / N_ball
    double alpha[4];    // bilinear corner weights: (l,l), (l,l+1), (l+1,l), (l+1,l+1)
    int g2_model;
    int hs_on;          // hard-sphere term on
    // External interaction force (collide without the shell sum):
    // C1 = fscale * fext + fdelta, both [3][N] FP32, either may be null.
    const float *fext;
    const float *fdelta;
    double fscale;
    // Mean-field attraction potential [N] (node order, no padding), or null:
    // the force gains -n (phi(r + e_a) - phi(r - e_a)) / 2.
    const double *phi;
    // Solid mask, or null: links[N] has bit i set when the node's neighbour
    // along c_i is solid, and LINK_SOLID when the node itself is; chi_n[N] is
    // then the per-node wall factor.
    const uint32_t *links;
    const double *chi_n;
};

constexpr uint32_t LINK_SOLID = 1u << 31;

// Separable weights of the mean-field attraction: w[m + R] = exp(-m^2 /
// range^2) for |m| <= R, and the depth eps.
constexpr int ATT_MAX_R = 30;
struct AttWeights {
    int R;
    double eps;
    double w[2 * ATT_MAX_R + 1];
};

template <typename TM>
struct Fields {
    TM *n;          // [fld_stride]
    TM *nj;         // [fld_stride][4]: (n, jx, jy, jz) interleaved, one load per shell read
    TM *eb;         // [fld_stride]
    TM *G;          // [7][fld_stride]
    TM *T;          // [fld_stride] temperature (thermal 39-velocity contexts), else null
};

// One slit of a batched ensemble.  Its populations start at pop_off in arrays
// of stride L.pop_stride shared by all slits, its padded fields at fld_off in
// arrays of stride L.fld_stride, its wall-factor table at chi_off.
struct SlitDesc {
    LatticeDev L;
    StepConst sc;
    int sigma;
    int pop_off;
    int fld_off;
    int chi_off;
};

// Work item of a persistent batch kernel: (slit, block of 256 indices).
struct WorkItem {
    int slit;
    int block;
};

// Host-side launchers (hslb_kernels.hip).  All are asynchronous on `s`.
// Local equilibrium of (n, u) as full FP64 populations [19][N].
hipError_t launch_feq(hipStream_t s, const LatticeDev &L, const double *n, const double *u, double *out);
// Layer means [nz][19] of populations with stride `stride`, plus ref (if any).
template <typename TF>
hipError_t launch_layer_means(hipStream_t s, const LatticeDev &L, const TF *f, int stride, const double *ref,
                              double *out);
template <typename TF, typename TM>
hipError_t launch_moments(hipStream_t s, const LatticeDev &L, const double *nref, const TF *f,
                          Fields<TM> fld);
template <typename TM>
hipError_t launch_gfield(hipStream_t s, const LatticeDev &L, int g2_model, Fields<TM> fld);
// Moments plus the row sums of the two-pass ball sum in one launch; returns
// hipErrorInvalidValue (launching nothing) unless nx divides 256 and the plane
// is a multiple of 256.  Then launch_ballsum completes eta_bar.  write_n: also
// the separate density field fld.n (the interleaved (n, j) is always written;
// within a step only the attraction reads fld.n).
template <typename TF, typename TM>
hipError_t launch_moments_rs(hipStream_t s, const LatticeDev &L, int sigma, const double *nref, const TF *f,
                             Fields<TM> fld, TM *rs, bool write_n);
template <typename TM>
hipError_t launch_ballsum(hipStream_t s, const LatticeDev &L, int sigma, double eta_pref, Fields<TM> fld,
                          const TM *rs);
// Two-pass ball sum; rs holds (sigma/2 + 1) padded fields of row sums.
template <typename TM>
hipError_t launch_smooth2(hipStream_t s, const LatticeDev &L, int sigma, double eta_pref, Fields<TM> fld,
                          TM *rs);

// tiles: with FP32 storage and fields, nx a multiple of 64 and ny of 4, no
// solid mask, the hard-sphere force on and sigma in 2..8, the collide stages
// shell fields of each 64 x 4 tile through LDS (bit for bit the same result).
template <typename TF, typename TM>
hipError_t launch_collide(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c,
                          const double *chi, const TF *fin, TF *fout, Fields<TM> fld, bool tiles = false);
// Whether launch_collide with tiles = true takes the LDS-staged kernel.
bool collide_tiles_apply(const LatticeDev &L, int sigma, const StepConst &c, bool fp32);
template <typename TF, typename TM>
hipError_t launch_force(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c,
                        const double *chi, const TF *f, Fields<TM> fld, double *F);
template <typename TF>
hipError_t launch_profiles_pop(hipStream_t s, const LatticeDev &L, const double *nref, const TF *f,
                               double *out);
template <typename TM>
hipError_t launch_unpad(hipStream_t s, const LatticeDev &L, const TM *src, double *dst);
template <typename TF>
hipError_t launch_export_moments(hipStream_t s, const LatticeDev &L, const double *nref, const TF *f,
                                 double *n, double *u);
template <typename TF>
hipError_t launch_get_pop(hipStream_t s, const LatticeDev &L, const double *nref, const TF *f,
                          double *out);
template <typename TF>
hipError_t launch_set_pop(hipStream_t s, const LatticeDev &L, const double *nref, const double *in,
                          TF *f);

hipError_t launch_copy(hipStream_t s, const void *src, void *dst, size_t bytes);

// The 39-velocity lattice (FP64 populations [39][pop_stride], stored as they
// are, without a reference table).  feq: third-order equilibrium of (n, u) as
// [39][N] (0 on solid layers); moments: n and (n, j) into the padded fields;
// collide: force, regularised collision and streaming, one launch over the
// fluid layers; force: F[3][N] of the current fields; export: n[N], u[3][N].
// thermal: the non-isothermal terms (temperature field in fld.T, the
// temperature term of C^(1), the energy source C^(2), the thermal equilibrium
// and the second-order sources).  feq39 takes T[N] (null: the lattice
// temperature); force39 also writes C^(2) to Q[N] when Q is not null.
hipError_t launch_feq39(hipStream_t s, const LatticeDev &L, const double *n, const double *u, const double *T,
                        double *out);
hipError_t launch_moments39(hipStream_t s, const LatticeDev &L, const double *f, Fields<double> fld, bool thermal);
// The same fused with the ball sum's row sums (as launch_moments_rs: nx divides
// 256 and the plane is a multiple of 256, else hipErrorInvalidValue).
hipError_t launch_moments39_rs(hipStream_t s, const LatticeDev &L, int sigma, const double *f, Fields<double> fld,
                               bool thermal, double *rs);
hipError_t launch_collide39(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c, const double *chi,
                            const double *fin, double *fout, Fields<double> fld, bool thermal);
hipError_t launch_force39(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c, const double *chi,
                          const double *f, Fields<double> fld, bool thermal, double *F, double *Q);
hipError_t launch_export39(hipStream_t s, const LatticeDev &L, const double *f, double *n, double *u);
// Layer profiles [5][nz] as launch_profiles_pop.
hipError_t launch_profiles39(hipStream_t s, const LatticeDev &L, const double *f, double *out);

// a[k] = (double)(float)a[k]: FP32-representable reference tables, so that a
// solid node (all populations 0) is stored exactly as -ref in FP32.
hipError_t launch_round_f32(hipStream_t s, double *a, int count);

// Mean-field attraction potential of the padded density field n over all nz
// layers, as three passes along x, y and z (a and b hold the partial sums,
// [N] each): phi = -eps sum_o w(o_x) w(o_y) w(o_z) n(r + o).
template <typename TM>
hipError_t launch_attraction(hipStream_t s, const LatticeDev &L, const AttWeights &aw, const TM *n, double *a,
                             double *b, double *phi);

// Device-resident scratch of the allocation-free force entry point: a
// file-scope array of kScratchBytes on every GPU the library runs on.
// scratch_address sets *ptr to its device address on the current device
// (looked up with hipGetSymbolAddress once per device).  launch_fill sets
// count doubles to v; launch_chi writes the wall factor table chi[nz] of a
// lattice (1 on periodic z or with wall_reg 0).
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_address(void **ptr);
hipError_t launch_fill(hipStream_t s, double *a, size_t count, double v);
hipError_t launch_chi(hipStream_t s, const LatticeDev &L, int sigma, int wall_reg, double *chi);

// Batched ensemble: one persistent launch per phase over a work list.
// phase 0 moments, 1 row sums, 2 ball sums, 3 contact values, 4 moments with
// the row sums (phases 0 and 1 in one; only when every slit's layer is a whole
// number of 256-node blocks of whole x-rows) (the collide phase is
// launch_batch_collide).  rows16: every slit is 16 nodes wide in x.
template <typename TF, typename TM>
hipError_t launch_batch_phase(hipStream_t s, int phase, unsigned grid, const SlitDesc *desc,
                              const WorkItem *work, int nwork, const TF *fin, TF *fout, Fields<TM> fld,
                              TM *rs, const double *chi, bool rows16);
// Collide phase of every slit: work holds the fluid items.  rows16: every slit
// is 16 nodes wide in x (the shell sum then shares x-neighbour reads between
// the lanes of each 16-lane row).
template <typename TF, typename TM>
hipError_t launch_batch_collide(hipStream_t s, unsigned grid, const SlitDesc *desc, const WorkItem *work, int nwork,
                                const TF *fin, TF *fout, Fields<TM> fld, const double *chi, bool rows16);
// Layer profiles of every slit: items (slit, z); out holds 5 rows per slit
// layer at prof_off[slit] (n_z, u_z[3], sum n).
template <typename TF>
hipError_t launch_batch_profiles(hipStream_t s, const SlitDesc *desc, const WorkItem *items, int nitems,
                                 const int *prof_off, const TF *f, double *out);
// Layer means of every slit's stored populations into its write table.
template <typename TF>
hipError_t launch_batch_layer_means(hipStream_t s, const SlitDesc *desc, const WorkItem *items, int nitems,
                                    const TF *f);

}  // namespace hslb
