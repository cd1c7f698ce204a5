// Internal declarations shared by the host engine and the HIP kernels of
// libhslb.so.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hslb {

constexpr int NQ = 19;
constexpr int NGSLOT = 7;  // contact-value sub-lattices: bits x=1, y=2, z=4 (0..6)

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
    double n_ref;       // populations are stored as f_i - w_i n_ref
    double pref;        // -v_T^2 sigma^2 4 pi
    double kappa;       // 2 / (v_T sqrt(pi))
    double eta_pref;    // (pi sigma^3 / 6) / N_ball
    double alpha[4];    // bilinear corner weights: (l,l), (l,l+1), (l+1,l), (l+1,l+1)
    int g2_model;
    int hs_on;          // hard-sphere term on
};

template <typename TM>
struct Fields {
    TM *n;          // [fld_stride]
    TM *j;          // [3][fld_stride]
    TM *eb;         // [fld_stride]
    TM *G;          // [7][fld_stride]
};

// Host-side launchers (hslb_kernels.hip).  All are asynchronous on `s`.
template <typename TF>
hipError_t launch_init(hipStream_t s, const LatticeDev &L, double n_ref, const double *n,
                       const double *u, TF *f);
template <typename TF, typename TM>
hipError_t launch_moments(hipStream_t s, const LatticeDev &L, double n_ref, const TF *f,
                          Fields<TM> fld);
template <typename TM>
hipError_t launch_smooth(hipStream_t s, const LatticeDev &L, int sigma, double eta_pref,
                         Fields<TM> fld);
template <typename TM>
hipError_t launch_gfield(hipStream_t s, const LatticeDev &L, int g2_model, Fields<TM> fld);
// Two-pass ball sum; rs holds (sigma/2 + 1) padded fields of row sums.
template <typename TM>
hipError_t launch_smooth2(hipStream_t s, const LatticeDev &L, int sigma, double eta_pref, Fields<TM> fld,
                          TM *rs);

template <typename TF, typename TM>
hipError_t launch_collide(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c,
                          const double *chi, const TF *fin, TF *fout, Fields<TM> fld);
template <typename TF, typename TM>
hipError_t launch_force(hipStream_t s, const LatticeDev &L, int sigma, const StepConst &c,
                        const double *chi, const TF *f, Fields<TM> fld, double *F);
template <typename TF>
hipError_t launch_profiles_pop(hipStream_t s, const LatticeDev &L, double n_ref, const TF *f,
                               double *out);
template <typename TM>
hipError_t launch_unpad(hipStream_t s, const LatticeDev &L, const TM *src, double *dst);
template <typename TF>
hipError_t launch_export_moments(hipStream_t s, const LatticeDev &L, double n_ref, const TF *f,
                                 double *n, double *u);
template <typename TF>
hipError_t launch_get_pop(hipStream_t s, const LatticeDev &L, double n_ref, const TF *f,
                          double *out);
template <typename TF>
hipError_t launch_set_pop(hipStream_t s, const LatticeDev &L, double n_ref, const double *in,
                          TF *f);

hipError_t launch_copy(hipStream_t s, const void *src, void *dst, size_t bytes);

}  // namespace hslb
