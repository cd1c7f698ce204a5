// Host engine and C ABI of libhslb.so (declared in include/hslb.h).
//
// The engine owns every device buffer of one lattice, builds the per-sigma
// constants in FP64 on the host, sequences the kernels of a time step on one
// HIP stream, replays pairs of steps from captured HIP graphs, and copies
// results out on request.
#include "hslb.h"
#include "hslb_cnn.hpp"
#include "hslb_internal.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <cstdlib>
#include <map>
#include <memory>
#include <string>
#include <type_traits>

#include <vector>

// Steps per replay of the long graphs of a single lattice (even; 0 or 2: the
// two-step graphs only).  16 steps per replay took the benchmark slit's step
// from 68.7 to 67.2 us; the two-step graphs cover what remains before a
// reference refresh.
#ifndef HSLB_GRAPH_LONG
#define HSLB_GRAPH_LONG 16
#endif

// Default watchdog of a single lattice: finite state and total mass within
// 1e-3 of its initial value, checked every 1000 steps.
constexpr int64_t kWatchEvery = 1000;
constexpr double kWatchTol = 1e-3;

using namespace hslb;

namespace {

// ------------------------------------------------ distance to solid nodes

constexpr double kEdtInf = 1e30;

// Lower envelope of parabolas (Felzenszwalb and Huttenlocher's distance
// transform) along one line of m samples: out[q] = min_p f[p] + (q - p)^2
// over the p with f[p] < kEdtInf (kEdtInf everywhere when there is none).
void edt_line(const double *f, int m, double *out, std::vector<int> &v, std::vector<double> &zb)
{
    v.resize(m);
    zb.resize(m + 1);
    int k = -1;
    for (int q = 0; q < m; ++q) {
        if (f[q] >= kEdtInf) continue;
        if (k < 0) {
            k = 0;
            v[0] = q;
            zb[0] = -kEdtInf;
            zb[1] = kEdtInf;
            continue;
        }
        double s;
        while (true) {
            const int p = v[k];
            s = ((f[q] + (double)q * q) - (f[p] + (double)p * p)) / (2.0 * (q - p));
            if (s > zb[k] || k == 0) break;
            --k;
        }
        if (s <= zb[k]) {  // only for k == 0: the new parabola is lower everywhere
            v[0] = q;
            zb[1] = kEdtInf;
            continue;
        }
        ++k;
        v[k] = q;
        zb[k] = s;
        zb[k + 1] = kEdtInf;
    }
    if (k < 0) {
        for (int q = 0; q < m; ++q) out[q] = kEdtInf;
        return;
    }
    int j = 0;
    for (int q = 0; q < m; ++q) {
        while (zb[j + 1] < q) ++j;
        const double d = (double)(q - v[j]);
        out[q] = d * d + f[v[j]];
    }
}

// Squared Euclidean distance from every node to the nearest solid node centre
// (periodic images along x, y and, if zper, z), by one line transform per
// axis; a periodic line is transformed as three copies and read in the middle.
void solid_distance2(const std::vector<uint8_t> &sol, int nx, int ny, int nz, bool zper, std::vector<double> &d2)
{
    const int N = nx * ny * nz;
    d2.assign(N, kEdtInf);
    for (int id = 0; id < N; ++id)
        if (sol[id]) d2[id] = 0.0;
    std::vector<int> v;
    std::vector<double> zb, in, out;
    auto axis = [&](int n, bool per, int count, auto index) {
        const int m = per ? 3 * n : n;
        in.resize(m);
        out.resize(m);
        for (int l = 0; l < count; ++l) {
            for (int q = 0; q < m; ++q) in[q] = d2[index(l, q % n)];
            edt_line(in.data(), m, out.data(), v, zb);
            for (int q = 0; q < n; ++q) d2[index(l, q)] = out[per ? q + n : q];
        }
    };
    axis(nx, true, ny * nz, [&](int l, int q) { return q + nx * l; });
    axis(ny, true, nx * nz, [&](int l, int q) { return (l % nx) + nx * (q + ny * (l / nx)); });
    axis(nz, zper, nx * ny, [&](int l, int q) { return l + nx * ny * q; });
}

struct KernelTimer {
    bool enabled = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<std::string, std::pair<int, int>>> pending;  // name, (ev0, ev1)
    size_t used = 0;
    std::map<std::string, std::pair<double, int64_t>> totals;

    ~KernelTimer()
    {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
    hipError_t ev(hipEvent_t *out)
    {
        if (used == pool.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            pool.push_back(e);
        }
        *out = pool[used++];
        return hipSuccess;
    }
};

class Engine {
public:
    virtual ~Engine() = default;
    virtual int init(const double *n, const double *u) = 0;
    virtual int step(int64_t nsteps) = 0;
    virtual int moments(double *n, double *u) = 0;
    virtual int profiles(double *nz, double *uz) = 0;
    virtual int force(double *F) = 0;
    virtual int eta_bar(double *eb) = 0;
    virtual int attraction_potential(double *phi) = 0;
    virtual int set_solid(const uint8_t *solid)
    {
        (void)solid;
        return fail_state("not available on a batch");
    }
    virtual int get_pop(double *f) = 0;
    virtual int set_pop(const double *f) = 0;
    // thermal 39-velocity contexts only
    virtual int init_thermal(const double *n, const double *u, const double *T)
    {
        (void)n, (void)u, (void)T;
        return fail_state("not a thermal context");
    }
    virtual int thermal_fields(double *T, double *Q)
    {
        (void)T, (void)Q;
        return fail_state("not a thermal context");
    }
    virtual int sync() = 0;
    // Capture every HIP graph a later step replays, without running it.
    virtual int prepare() { return HSLB_OK; }
    virtual int timings(double *ms, double *mlups) = 0;
    virtual void set_stream(hipStream_t s) = 0;
    // batched ensembles only
    virtual int batch_init(int slit, const double *n, const double *u)
    {
        (void)slit, (void)n, (void)u;
        return fail_state("not a batch context");
    }
    virtual int batch_profiles(int slit, double *nz, double *uz)
    {
        (void)slit, (void)nz, (void)uz;
        return fail_state("not a batch context");
    }
    virtual int batch_finite(int32_t *flags)
    {
        (void)flags;
        return fail_state("not a batch context");
    }
    virtual int batch_autotune(int32_t steps, int32_t *choice, double *us_per_step, int32_t cap)
    {
        (void)steps, (void)choice, (void)us_per_step, (void)cap;
        return fail_state("not a batch context");
    }
    virtual int batch_set_config(int32_t grid_per_cu, int32_t order)
    {
        (void)grid_per_cu, (void)order;
        return fail_state("not a batch context");
    }
    virtual int batch_set_launch(int32_t phase_grid, int32_t collide_grid, int32_t order)
    {
        (void)phase_grid, (void)collide_grid, (void)order;
        return fail_state("not a batch context");
    }
    virtual int batch_get_launch(int32_t *phase_grid, int32_t *collide_grid, int32_t *order)
    {
        (void)phase_grid, (void)collide_grid, (void)order;
        return fail_state("not a batch context");
    }
    virtual int checkpoint_bytes(int64_t *bytes)
    {
        (void)bytes;
        return fail_state("checkpoints are per lattice");
    }
    virtual int checkpoint_save(void *buf)
    {
        (void)buf;
        return fail_state("checkpoints are per lattice");
    }
    virtual int checkpoint_load(const void *buf)
    {
        (void)buf;
        return fail_state("checkpoints are per lattice");
    }
    // learned force (single lattices only)
    virtual int surr_set_weights(const float *w) { (void)w; return fail_state("learned force needs a single lattice"); }
    virtual int surr_get_weights(float *w) { (void)w; return fail_state("learned force needs a single lattice"); }
    virtual int surr_set_mode(int mode) { (void)mode; return fail_state("learned force needs a single lattice"); }
    virtual int surr_set_components(int mask) { (void)mask; return fail_state("learned force needs a single lattice"); }
    virtual int surr_stats(int64_t *checks, int64_t *fallback, double *last_r, double *max_r)
    {
        (void)checks, (void)fallback, (void)last_r, (void)max_r;
        return fail_state("learned force needs a single lattice");
    }
    virtual int surr_force(double *F) { (void)F; return fail_state("learned force needs a single lattice"); }
    // network input x = bf16(eta) and target C1 / force scale of the current state
    virtual int training_pair(uint16_t *x, float *target, cnn::Geo *g, int *wall_lo, int *wall_hi, int *sigma)
    {
        (void)x, (void)target, (void)g, (void)wall_lo, (void)wall_hi, (void)sigma;
        return fail_state("training pairs come from single lattices");
    }
    int fail_state(const char *msg)
    {
        err = msg;
        return HSLB_ESTATE;
    }
    std::string err;
    int64_t steps = 0;
    bool inited = false;
    int64_t watch_every = 0;
    double watch_tol = 0.0;
    bool use_graph = true;
    // collide with shell fields staged through LDS where the lattice allows
    // (off by default: it measured no faster than the direct reads)
    virtual int set_collide_tiles(bool on)
    {
        collide_tiles = on;
        return HSLB_OK;
    }
    bool collide_tiles = false;
    int64_t shift_every = 0;  // refresh period of the layer reference densities (0: never)
    KernelTimer kt;
};

int fail(std::string &err, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return code;
}

#define HIP_TRY(...)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (__VA_ARGS__);                                                             \
        if (e_ != hipSuccess)                                                                      \
            return fail(err, HSLB_EDEVICE, "%s failed: %s", #__VA_ARGS__, hipGetErrorString(e_));  \
    } while (0)

int ball_count(int sigma)
{
    int r = sigma / 2 + 1, c = 0;
    for (int z = -r; z <= r; ++z)
        for (int y = -r; y <= r; ++y)
            for (int x = -r; x <= r; ++x)
                if (4 * (x * x + y * y + z * z) <= sigma * sigma) ++c;
    return c;
}

template <typename TF, typename TM>
class EngineT final : public Engine {
public:
    EngineT(const hslb_params &p) : p_(p) {}

    ~EngineT() override
    {
        for (int k = 0; k < 2; ++k) {
            if (gexec_[k]) (void)hipGraphExecDestroy(gexec_[k]);
            if (gexecL_[k]) (void)hipGraphExecDestroy(gexecL_[k]);
        }
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
        (void)hipFree(f_[0]);
        (void)hipFree(f_[1]);
        (void)hipFree(fld_mem_);
        (void)hipFree(chi_d_);
        (void)hipFree(att_d_);
        (void)hipFree(links_d_);
        (void)hipFree(chi_n_d_);
        (void)hipFree(prof_d_);
        (void)hipFree(nref_d_);
        (void)hipHostFree(prof_h_);
        (void)hipFree(io_d_);
        (void)hipFree(surr_mem_);
        (void)hipHostFree(jpart_h_);
        if (own_stream_ && stream_) (void)hipStreamDestroy(stream_);
    }

    int setup()
    {
        const int sig = p_.sigma >= 2 ? p_.sigma : 2;
        L_.nx = p_.nx;
        L_.ny = p_.ny;
        L_.nz = p_.nz;
        L_.wall_lo = p_.wall_lo;
        L_.wall_hi = p_.wall_hi;
        L_.zper = (p_.wall_lo == 0 && p_.wall_hi == 0) ? 1 : 0;
        L_.hz = sig;
        L_.plane = p_.nx * p_.ny;
        L_.N = L_.plane * p_.nz;
        L_.pop_stride = (L_.N + 63) / 64 * 64;
        L_.fld_stride = (L_.plane * (p_.nz + 2 * L_.hz) + 63) / 64 * 64;
        sigma_ = sig;
        q_ = (p_.lattice == HSLB_D3Q39) ? Q39 : NQ;
        thermal_ = (p_.thermal == 1);

        sc_.tau = p_.tau;
        for (int a = 0; a < 3; ++a) sc_.g[a] = p_.accel[a];
        const double vt2 = l39() ? CS2_39 : 1.0 / 3.0;
        sc_.pref = -vt2 * (double)sig * (double)sig * 4.0 * M_PI;
        sc_.kappa = 2.0 / (std::sqrt(vt2) * std::sqrt(M_PI));
        sc_.eta_pref = M_PI * (double)sig * sig * sig / 6.0 / (double)ball_count(sig);
        const double A = (double)sig / std::sqrt(2.0);
        const double th = A - std::floor(A);
        sc_.alpha[0] = (1.0 - th) * (1.0 - th);
        sc_.alpha[1] = (1.0 - th) * th;
        sc_.alpha[2] = th * (1.0 - th);
        sc_.alpha[3] = th * th;
        sc_.g2_model = p_.g2_model;
        sc_.hs_on = (p_.force_mode == HSLB_FORCE_OFF) ? 0 : 1;

        HIP_TRY(hipStreamCreate(&stream_));
        own_stream_ = true;
        HIP_TRY(hipEventCreate(&ev0_));
        HIP_TRY(hipEventCreate(&ev1_));
        const size_t popb = sizeof(TF) * (size_t)q_ * L_.pop_stride;
        if (hipMalloc(&f_[0], popb) != hipSuccess || hipMalloc(&f_[1], popb) != hipSuccess)
            return fail(err, HSLB_ENOMEM, "population buffers (%zu bytes each) do not fit", popb);
        // n, j, eta_bar, the 7 contact-value slots and sigma/2 + 1 row-sum fields
        // (plus the temperature in thermal contexts)
        const size_t nfld = (size_t)(1 + 4 + 1 + NGSLOT + sig / 2 + 1 + (thermal_ ? 1 : 0)) * L_.fld_stride;
        if (hipMalloc(&fld_mem_, sizeof(TM) * nfld) != hipSuccess)
            return fail(err, HSLB_ENOMEM, "moment fields do not fit");
        HIP_TRY(hipMemset(fld_mem_, 0, sizeof(TM) * nfld));
        HIP_TRY(hipMemset(f_[0], 0, popb));
        HIP_TRY(hipMemset(f_[1], 0, popb));
        fld_.n = fld_mem_;
        fld_.nj = fld_mem_ + L_.fld_stride;
        fld_.eb = fld_mem_ + 5 * (size_t)L_.fld_stride;
        fld_.G = fld_mem_ + 6 * (size_t)L_.fld_stride;
        rs_ = fld_mem_ + (size_t)(6 + NGSLOT) * L_.fld_stride;
        fld_.T = thermal_ ? rs_ + (size_t)(sig / 2 + 1) * L_.fld_stride : nullptr;

        std::vector<double> chi(p_.nz, 1.0);
        if (!L_.zper && p_.wall_reg) {
            const double za = p_.wall_lo - 0.5, zb = p_.nz - p_.wall_hi - 0.5;
            for (int z = 0; z < p_.nz; ++z) {
                const double dw = std::fmin((double)z - za, zb - (double)z);
                chi[z] = 1.0 - std::exp(-dw / (double)sig);
            }
        }
        if (p_.att_eps != 0.0) {
            aw_.R = (int)std::ceil(3.0 * p_.att_range);
            aw_.eps = p_.att_eps;
            for (int m = -aw_.R; m <= aw_.R; ++m)
                aw_.w[m + aw_.R] = std::exp(-(double)(m * m) / (p_.att_range * p_.att_range));
            if (hipMalloc(&att_d_, sizeof(double) * 3 * (size_t)L_.N) != hipSuccess)
                return fail(err, HSLB_ENOMEM, "attraction fields do not fit");
            HIP_TRY(hipMemset(att_d_, 0, sizeof(double) * 3 * (size_t)L_.N));
            sc_.phi = att_d_ + 2 * (size_t)L_.N;
        }
        HIP_TRY(hipMalloc(&chi_d_, sizeof(double) * p_.nz));
        HIP_TRY(hipMemcpy(chi_d_, chi.data(), sizeof(double) * p_.nz, hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc(&prof_d_, sizeof(double) * 5 * p_.nz));
        HIP_TRY(hipMalloc(&nref_d_, sizeof(double) * 2 * NQ * p_.nz));
        HIP_TRY(hipMemset(nref_d_, 0, sizeof(double) * 2 * NQ * p_.nz));
        sc_.nref_r = nref_d_;
        sc_.nref_w = nref_d_ + NQ * p_.nz;
        shift_every = (sizeof(TF) == 4) ? 50 : 0;
        HIP_TRY(hipHostMalloc((void **)&prof_h_, sizeof(double) * 5 * p_.nz, hipHostMallocDefault));
        return HSLB_OK;
    }

    void set_stream(hipStream_t s) override { ext_stream_ = s; }

    hipStream_t st() const { return ext_stream_ ? ext_stream_ : stream_; }

    bool fluid_z(int z) const { return L_.zper || (z >= L_.wall_lo && z < L_.nz - L_.wall_hi); }

    int io(size_t bytes, double **out)
    {
        if (bytes > io_bytes_) {
            (void)hipFree(io_d_);
            io_d_ = nullptr;
            io_bytes_ = 0;
            if (hipMalloc(&io_d_, bytes) != hipSuccess) return fail(err, HSLB_ENOMEM, "staging buffer");
            io_bytes_ = bytes;
        }
        *out = io_d_;
        return HSLB_OK;
    }

    int set_collide_tiles(bool on) override
    {
        if (on != collide_tiles) drop_graphs();  // the captured steps hold the other kernel
        collide_tiles = on;
        return HSLB_OK;
    }

    void drop_graphs()
    {
        for (int k = 0; k < 2; ++k) {
            if (gexec_[k]) {
                (void)hipGraphExecDestroy(gexec_[k]);
                gexec_[k] = nullptr;
            }
            if (gexecL_[k]) {
                (void)hipGraphExecDestroy(gexecL_[k]);
                gexecL_[k] = nullptr;
            }
        }
    }

    // Store full FP64 populations [19][N] (device): the reference tables
    // become their layer means, then the populations are stored relative to them.
    // With a solid mask and FP32 storage, reference tables are rounded to
    // FP32 so that a solid node's zero populations are stored exactly (-ref).
    int round_refs(double *table)
    {
        if (sc_.links && sizeof(TF) == 4) HIP_TRY(launch_round_f32(st(), table, NQ * L_.nz));
        return HSLB_OK;
    }

    int store_populations(const double *stage)
    {
        if (l39()) {
            // FP64 storage as given: [39][N] into the padded [39][pop_stride]
            if constexpr (!std::is_same<TF, double>::value) return fail(err, HSLB_EINVAL, "D3Q39 is FP64 only");
            HIP_TRY(hipMemcpy2DAsync(f_[cur_], sizeof(double) * L_.pop_stride, stage, sizeof(double) * L_.N,
                                     sizeof(double) * L_.N, Q39, hipMemcpyDeviceToDevice, st()));
            return HSLB_OK;
        }
        HIP_TRY(launch_layer_means<double>(st(), L_, stage, L_.N, nullptr, nref_d_));
        int rc = round_refs(nref_d_);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(nref_d_ + NQ * L_.nz, nref_d_, sizeof(double) * NQ * L_.nz, hipMemcpyDeviceToDevice,
                               st()));
        HIP_TRY(launch_set_pop<TF>(st(), L_, nref_d_, stage, f_[cur_]));
        return HSLB_OK;
    }

    int init(const double *n, const double *u) override { return init_fields(n, u, nullptr); }

    int init_thermal(const double *n, const double *u, const double *T) override
    {
        if (!thermal_) return fail(err, HSLB_ESTATE, "not a thermal context");
        return init_fields(n, u, T);
    }

    int init_fields(const double *n, const double *u, const double *T)
    {
        const int N = L_.N;
        std::vector<double> nm, um;
        if (!solid_h_.empty()) {
            // solid nodes carry nothing
            nm.assign(n, n + N);
            if (u) um.assign(u, u + 3 * (size_t)N);
            for (int id = 0; id < N; ++id)
                if (solid_h_[id]) {
                    nm[id] = 0.0;
                    if (u)
                        for (int a = 0; a < 3; ++a) um[(size_t)a * N + id] = 0.0;
                }
            n = nm.data();
            if (u) u = um.data();
        }
        double msum = 0.0;
        int64_t nfl = 0;
        for (int id = 0; id < N; ++id) {
            if (!fluid_z(id / L_.plane)) continue;
            if (!std::isfinite(n[id]) || n[id] < 0.0)
                return fail(err, HSLB_EINVAL, "density at node %d is negative or not finite", id);
            if (u)
                for (int a = 0; a < 3; ++a)
                    if (!std::isfinite(u[(size_t)a * N + id]))
                        return fail(err, HSLB_EINVAL, "velocity at node %d is not finite", id);
            if (T && !(std::isfinite(T[id]) && T[id] > 0.0))
                return fail(err, HSLB_EINVAL, "temperature at node %d is not positive and finite", id);
            msum += n[id];
            ++nfl;
        }
        mass0_ = msum;
        double *d;
        int rc = io(sizeof(double) * (5 + q_) * (size_t)N, &d);
        if (rc) return rc;
        double *stage = d + 5 * (size_t)N;
        if (T) HIP_TRY(hipMemcpyAsync(d + 4 * (size_t)N, T, sizeof(double) * N, hipMemcpyHostToDevice, st()));
        HIP_TRY(hipMemcpyAsync(d, n, sizeof(double) * N, hipMemcpyHostToDevice, st()));
        if (u)
            HIP_TRY(hipMemcpyAsync(d + N, u, sizeof(double) * 3 * (size_t)N, hipMemcpyHostToDevice, st()));
        else
            HIP_TRY(hipMemsetAsync(d + N, 0, sizeof(double) * 3 * (size_t)N, st()));
        cur_ = 0;
        if (l39())
            HIP_TRY(launch_feq39(st(), L_, d, d + N, T ? d + 4 * (size_t)N : nullptr, stage));
        else
            HIP_TRY(launch_feq(st(), L_, d, d + N, stage));
        rc = store_populations(stage);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(st()));
        drop_graphs();
        steps = 0;
        refreshed_at_ = -1;
        inited = true;
        surr_ok_ = false;
        have_delta_ = false;
        return HSLB_OK;
    }

    // Launch one kernel, bracketed by timing events when enabled.
    template <typename Fn>
    int launch(const char *name, Fn &&fn)
    {
        hipEvent_t a = nullptr, b = nullptr;
        if (kt.enabled && !capturing_) {
            HIP_TRY(kt.ev(&a));
            HIP_TRY(kt.ev(&b));
            HIP_TRY(hipEventRecord(a, st()));
        }
        HIP_TRY(fn());
        if (a) {
            HIP_TRY(hipEventRecord(b, st()));
            kt.pending.push_back({name, {(int)kt.used - 2, (int)kt.used - 1}});
        }
        return HSLB_OK;
    }

    // Coarse-grained density and contact values of the current moments.
    int fields_hs()
    {
        int rc = launch("smooth", [&] { return launch_smooth2<TM>(st(), L_, sigma_, sc_.eta_pref, fld_, rs_); });
        if (rc) return rc;
        return launch("gfield", [&] { return launch_gfield<TM>(st(), L_, sc_.g2_model, fld_); });
    }

    // whole x-rows per 256-thread block: moments and row sums in one launch
    bool fused_rows() const { return 256 % L_.nx == 0 && L_.plane % 256 == 0; }

    // Moments into the padded fields, for the readouts.
    hipError_t moments_fields()
    {
        if (l39()) return launch_moments39(st(), L_, (const double *)f_[cur_], fld39(), thermal_);
        return launch_moments<TF, TM>(st(), L_, nref_d_, f_[cur_], fld_);
    }

    // The fields as the 39-velocity kernels take them (FP64 contexts only).
    Fields<double> fld39() const
    {
        Fields<double> f{};
        if constexpr (std::is_same<TM, double>::value) f = fld_;
        return f;
    }

    int one_step39()
    {
        if constexpr (!std::is_same<TF, double>::value) {
            return fail(err, HSLB_EINVAL, "D3Q39 is FP64 only");
        } else {
            int rc;
            if (sc_.hs_on && fused_rows()) {
                double *rs = nullptr;
                if constexpr (std::is_same<TM, double>::value) rs = rs_;
                rc = launch("moments", [&] {
                    return launch_moments39_rs(st(), L_, sigma_, f_[cur_], fld39(), thermal_, rs);
                });
                if (rc) return rc;
                rc = launch("smooth", [&] { return launch_ballsum<TM>(st(), L_, sigma_, sc_.eta_pref, fld_, rs_); });
                if (rc) return rc;
                rc = launch("gfield", [&] { return launch_gfield<TM>(st(), L_, sc_.g2_model, fld_); });
                if (rc) return rc;
            } else {
                rc = launch("moments", [&] { return launch_moments39(st(), L_, f_[cur_], fld39(), thermal_); });
                if (rc) return rc;
                if (sc_.hs_on && (rc = fields_hs())) return rc;
            }
            if (sc_.phi && (rc = attraction())) return rc;
            rc = launch("collide", [&] {
                return launch_collide39(st(), L_, sigma_, sc_, chi_d_, f_[cur_], f_[1 - cur_], fld39(), thermal_);
            });
            if (rc) return rc;
            cur_ = 1 - cur_;
            return HSLB_OK;
        }
    }

    int one_step()
    {
        int rc;
        if (l39()) return one_step39();
        if (sc_.hs_on && fused_rows()) {
            rc = launch("moments", [&] {
                return launch_moments_rs<TF, TM>(st(), L_, sigma_, nref_d_, f_[cur_], fld_, rs_, sc_.phi != nullptr);
            });
            if (rc) return rc;
            rc = launch("smooth", [&] { return launch_ballsum<TM>(st(), L_, sigma_, sc_.eta_pref, fld_, rs_); });
            if (rc) return rc;
            rc = launch("gfield", [&] { return launch_gfield<TM>(st(), L_, sc_.g2_model, fld_); });
            if (rc) return rc;
        } else {
            rc = launch("moments", [&] { return launch_moments<TF, TM>(st(), L_, nref_d_, f_[cur_], fld_); });
            if (rc) return rc;
            if (sc_.hs_on && (rc = fields_hs())) return rc;
        }
        if (sc_.phi && (rc = attraction())) return rc;
        rc = launch("collide", [&] {
            return launch_collide<TF, TM>(st(), L_, sigma_, sc_, chi_d_, f_[cur_], f_[1 - cur_], fld_, collide_tiles);
        });
        if (rc) return rc;
        cur_ = 1 - cur_;
        return HSLB_OK;
    }

    // Mean-field attraction potential of the current moments (into sc_.phi).
    int attraction()
    {
        return launch("attract", [&] {
            return launch_attraction<TM>(st(), L_, aw_, fld_.n, att_d_, att_d_ + (size_t)L_.N,
                                         att_d_ + 2 * (size_t)L_.N);
        });
    }

    int capture(int parity, int len = 2)
    {
        const int save = cur_;
        cur_ = parity;
        hipGraph_t g = nullptr;
        capturing_ = true;
        HIP_TRY(hipStreamBeginCapture(st(), hipStreamCaptureModeThreadLocal));
        int rc = HSLB_OK;
        for (int k = 0; k < len && !rc; ++k) rc = one_step();
        hipGraph_t gg = nullptr;
        hipError_t e = hipStreamEndCapture(st(), &gg);
        capturing_ = false;
        cur_ = save;
        if (rc) {
            if (gg) (void)hipGraphDestroy(gg);
            return rc;
        }
        if (e != hipSuccess) return fail(err, HSLB_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        g = gg;
        e = hipGraphInstantiate(len == 2 ? &gexec_[parity] : &gexecL_[parity], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(err, HSLB_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
        return HSLB_OK;
    }

    int prepare() override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "prepare before init");
        if (!use_graph || kt.enabled || p_.force_mode == HSLB_FORCE_SURROGATE) return HSLB_OK;
        for (int par = 0; par < 2; ++par) {
            int rc = HSLB_OK;
            if (HSLB_GRAPH_LONG > 2 && !gexecL_[par]) rc = capture(par, HSLB_GRAPH_LONG);
            if (!rc && !gexec_[par]) rc = capture(par);
            if (rc) return rc;
        }
        return HSLB_OK;
    }

    // One step that moves the reference tables to the current layer means of
    // the populations: the step reads with the old table, writes with the new.
    int refresh_step()
    {
        HIP_TRY(launch_layer_means<TF>(st(), L_, f_[cur_], L_.pop_stride, nref_d_, nref_d_ + NQ * L_.nz));
        int rc = round_refs(nref_d_ + NQ * L_.nz);
        if (rc) return rc;
        rc = one_step();
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(nref_d_, nref_d_ + NQ * L_.nz, sizeof(double) * NQ * L_.nz, hipMemcpyDeviceToDevice,
                               st()));
        return HSLB_OK;
    }

    int advance(int64_t n)
    {
        if (p_.force_mode == HSLB_FORCE_SURROGATE) return advance_surrogate(n);
        const bool graph = use_graph && !kt.enabled;
        while (n > 0) {
            if (shift_every > 0 && steps > 0 && steps % shift_every == 0 && refreshed_at_ != steps) {
                int rc = refresh_step();
                if (rc) return rc;
                refreshed_at_ = steps;
                n -= 1;
                steps += 1;
                continue;
            }
            const int64_t room = shift_every > 0 ? shift_every - steps % shift_every : n;
            if (graph && HSLB_GRAPH_LONG > 2 && n >= HSLB_GRAPH_LONG && room >= HSLB_GRAPH_LONG) {
                if (!gexecL_[cur_]) {
                    int rc = capture(cur_, HSLB_GRAPH_LONG);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(gexecL_[cur_], st()));
                n -= HSLB_GRAPH_LONG;
                steps += HSLB_GRAPH_LONG;
            } else if (graph && n >= 2 && room >= 2) {
                if (!gexec_[cur_]) {
                    int rc = capture(cur_);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(gexec_[cur_], st()));
                n -= 2;
                steps += 2;
            } else {
                int rc = one_step();
                if (rc) return rc;
                n -= 1;
                steps += 1;
            }
        }
        return HSLB_OK;
    }

    int collect_kernel_times()
    {
        if (kt.pending.empty()) return HSLB_OK;
        HIP_TRY(hipStreamSynchronize(st()));
        for (auto &pr : kt.pending) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, kt.pool[pr.second.first], kt.pool[pr.second.second]));
            auto &t = kt.totals[pr.first];
            t.first += ms;
            t.second += 1;
        }
        kt.pending.clear();
        kt.used = 0;
        return HSLB_OK;
    }

    hipError_t launch_profiles()
    {
        if (l39()) return launch_profiles39(st(), L_, (const double *)f_[cur_], prof_d_);
        return launch_profiles_pop<TF>(st(), L_, nref_d_, f_[cur_], prof_d_);
    }

    int watchdog_check()
    {
        HIP_TRY(launch_profiles());
        HIP_TRY(hipMemcpyAsync(prof_h_, prof_d_, sizeof(double) * 5 * L_.nz, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        double m = 0.0;
        bool fin = true;
        for (int k = 0; k < 5 * L_.nz; ++k)
            if (!std::isfinite(prof_h_[k])) fin = false;
        for (int z = 0; z < L_.nz; ++z) m += prof_h_[4 * L_.nz + z];
        if (!fin) return fail(err, HSLB_EUNSTABLE, "non-finite state at step %lld", (long long)steps);
        if (mass0_ > 0 && std::fabs(m - mass0_) > watch_tol * mass0_)
            return fail(err, HSLB_EUNSTABLE, "mass drift %.3e at step %lld", (m - mass0_) / mass0_,
                        (long long)steps);
        return HSLB_OK;
    }

    int step(int64_t nsteps) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "step before init");
        if (nsteps < 0) return fail(err, HSLB_EINVAL, "negative step count");
        HIP_TRY(hipEventRecord(ev0_, st()));
        int64_t left = nsteps;
        while (left > 0) {
            int64_t chunk = left;
            if (watch_every > 0) {
                const int64_t to_check = watch_every - (steps % watch_every);
                chunk = std::min(left, to_check);
            }
            int rc = advance(chunk);
            if (rc) return rc;
            left -= chunk;
            if (watch_every > 0 && steps % watch_every == 0) {
                rc = watchdog_check();
                if (rc) return rc;
            }
        }
        HIP_TRY(hipEventRecord(ev1_, st()));
        last_steps_ = nsteps;
        if (kt.enabled) return collect_kernel_times();
        return HSLB_OK;
    }

    int sync() override
    {
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int timings(double *ms, double *mlups) override
    {
        HIP_TRY(hipEventSynchronize(ev1_));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, ev0_, ev1_));
        const double per = last_steps_ > 0 ? (double)t / (double)last_steps_ : 0.0;
        const double nfl = (double)L_.plane * (double)(L_.nz - L_.wall_lo - L_.wall_hi);
        if (ms) *ms = per;
        if (mlups) *mlups = per > 0 ? nfl / (per * 1e-3) / 1e6 : 0.0;
        return HSLB_OK;
    }

    int moments(double *n, double *u) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "moments before init");
        double *d;
        const size_t N = L_.N;
        int rc = io(sizeof(double) * 4 * N, &d);
        if (rc) return rc;
        if (l39())
            HIP_TRY(launch_export39(st(), L_, (const double *)f_[cur_], d, d + N));
        else
            HIP_TRY(launch_export_moments<TF>(st(), L_, nref_d_, f_[cur_], d, d + N));
        if (n) HIP_TRY(hipMemcpyAsync(n, d, sizeof(double) * N, hipMemcpyDeviceToHost, st()));
        if (u) HIP_TRY(hipMemcpyAsync(u, d + N, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int profiles(double *nz, double *uz) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "profiles before init");
        HIP_TRY(launch_profiles());
        HIP_TRY(hipMemcpyAsync(prof_h_, prof_d_, sizeof(double) * 5 * L_.nz, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        if (nz) std::memcpy(nz, prof_h_, sizeof(double) * L_.nz);
        if (uz) std::memcpy(uz, prof_h_ + L_.nz, sizeof(double) * 3 * L_.nz);
        return HSLB_OK;
    }

    int force(double *F) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "force before init");
        double *d;
        const size_t N = L_.N;
        int rc = io(sizeof(double) * 3 * N, &d);
        if (rc) return rc;
        HIP_TRY(moments_fields());
        if (sc_.hs_on && (rc = fields_hs())) return rc;
        if (sc_.phi && (rc = attraction())) return rc;
        if (l39())
            HIP_TRY(launch_force39(st(), L_, sigma_, sc_, chi_d_, (const double *)f_[cur_], fld39(), thermal_, d,
                                   nullptr));
        else
            HIP_TRY(launch_force<TF, TM>(st(), L_, sigma_, sc_, chi_d_, f_[cur_], fld_, d));
        HIP_TRY(hipMemcpyAsync(F, d, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int thermal_fields(double *T, double *Q) override
    {
        if (!thermal_) return fail(err, HSLB_ESTATE, "not a thermal context");
        if (!inited) return fail(err, HSLB_ESTATE, "thermal_fields before init");
        double *d;
        const size_t N = L_.N;
        int rc = io(sizeof(double) * 5 * N, &d);
        if (rc) return rc;
        HIP_TRY(moments_fields());
        if (sc_.hs_on && (rc = fields_hs())) return rc;
        if (sc_.phi && (rc = attraction())) return rc;
        HIP_TRY(launch_force39(st(), L_, sigma_, sc_, chi_d_, (const double *)f_[cur_], fld39(), true, d,
                               d + 3 * N));
        HIP_TRY(launch_unpad<TM>(st(), L_, fld_.T, d + 4 * N));
        if (T) HIP_TRY(hipMemcpyAsync(T, d + 4 * N, sizeof(double) * N, hipMemcpyDeviceToHost, st()));
        if (Q) HIP_TRY(hipMemcpyAsync(Q, d + 3 * N, sizeof(double) * N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int set_solid(const uint8_t *solid) override
    {
        if (inited) return fail(err, HSLB_ESTATE, "set_solid after init");
        if (l39()) return fail(err, HSLB_EINVAL, "solid masks are not available on the 39-velocity lattice");
        if (p_.force_mode == HSLB_FORCE_SURROGATE)
            return fail(err, HSLB_EINVAL, "solid masks are not available with the learned force");
        const int N = L_.N, nx = L_.nx, ny = L_.ny, nz = L_.nz;
        solid_h_.assign(N, 0);
        std::vector<uint8_t> sol(N);
        for (int id = 0; id < N; ++id) {
            solid_h_[id] = (solid[id] != 0 && fluid_z(id / L_.plane)) ? 1 : 0;
            sol[id] = (solid[id] != 0 || !fluid_z(id / L_.plane)) ? 1 : 0;
        }
        std::vector<uint32_t> links(N, 0u);
        for (int id = 0; id < N; ++id) {
            const int z = id / L_.plane, y = (id / nx) % ny, x = id % nx;
            if (sol[id]) {
                links[id] = LINK_SOLID;
                continue;
            }
            for (int i = 0; i < NQ; ++i) {
                const int xt = (x + CX[i] + nx) % nx, yt = (y + CY[i] + ny) % ny;
                int zt = z + CZ[i];
                if (L_.zper) zt = (zt + nz) % nz;
                if (zt < 0 || zt >= nz || sol[xt + nx * (yt + ny * zt)]) links[id] |= 1u << i;
            }
        }
        std::vector<double> chi(N, 1.0);
        if (p_.wall_reg) {
            std::vector<double> d2;
            solid_distance2(sol, nx, ny, nz, L_.zper != 0, d2);
            for (int id = 0; id < N; ++id)
                if (!sol[id] && d2[id] < kEdtInf)
                    chi[id] = 1.0 - std::exp(-(std::sqrt(d2[id]) - 0.5) / (double)sigma_);
        }
        if (!links_d_ && hipMalloc(&links_d_, sizeof(uint32_t) * N) != hipSuccess)
            return fail(err, HSLB_ENOMEM, "solid links do not fit");
        if (!chi_n_d_ && hipMalloc(&chi_n_d_, sizeof(double) * N) != hipSuccess)
            return fail(err, HSLB_ENOMEM, "wall factors do not fit");
        HIP_TRY(hipMemcpy(links_d_, links.data(), sizeof(uint32_t) * N, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(chi_n_d_, chi.data(), sizeof(double) * N, hipMemcpyHostToDevice));
        sc_.links = links_d_;
        sc_.chi_n = chi_n_d_;
        drop_graphs();
        return HSLB_OK;
    }

    int attraction_potential(double *phi) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "attraction_potential before init");
        if (!sc_.phi) {
            std::memset(phi, 0, sizeof(double) * (size_t)L_.N);
            return HSLB_OK;
        }
        HIP_TRY(moments_fields());
        int rc = attraction();
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(phi, sc_.phi, sizeof(double) * L_.N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int eta_bar(double *eb) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "eta_bar before init");
        double *d;
        int rc = io(sizeof(double) * (size_t)L_.N, &d);
        if (rc) return rc;
        HIP_TRY(moments_fields());
        HIP_TRY(launch_smooth2<TM>(st(), L_, sigma_, sc_.eta_pref, fld_, rs_));
        HIP_TRY(launch_unpad<TM>(st(), L_, fld_.eb, d));
        HIP_TRY(hipMemcpyAsync(eb, d, sizeof(double) * L_.N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int get_pop(double *f) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "get_populations before init");
        if (l39()) {
            HIP_TRY(hipMemcpy2DAsync(f, sizeof(double) * L_.N, f_[cur_], sizeof(TF) * L_.pop_stride,
                                     sizeof(double) * L_.N, Q39, hipMemcpyDeviceToHost, st()));
            HIP_TRY(hipStreamSynchronize(st()));
            return HSLB_OK;
        }
        double *d;
        const size_t tot = (size_t)NQ * L_.N;
        int rc = io(sizeof(double) * tot, &d);
        if (rc) return rc;
        HIP_TRY(launch_get_pop<TF>(st(), L_, nref_d_, f_[cur_], d));
        HIP_TRY(hipMemcpyAsync(f, d, sizeof(double) * tot, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int set_pop(const double *f) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "set_populations before init");
        const size_t tot = (size_t)q_ * L_.N;
        for (size_t k = 0; k < tot; ++k)
            if (!std::isfinite(f[k]))
                return fail(err, HSLB_EINVAL, "population %zu is not finite", k);
        std::vector<double> fm;
        if (l39()) {
            // solid layers carry nothing
            fm.assign(f, f + tot);
            for (int id = 0; id < L_.N; ++id)
                if (!fluid_z(id / L_.plane))
                    for (int i = 0; i < Q39; ++i) fm[(size_t)i * L_.N + id] = 0.0;
            f = fm.data();
        }
        if (!solid_h_.empty()) {
            fm.assign(f, f + tot);
            for (int id = 0; id < L_.N; ++id)
                if (solid_h_[id])
                    for (int i = 0; i < NQ; ++i) fm[(size_t)i * L_.N + id] = 0.0;
            f = fm.data();
        }
        double *d;
        int rc = io(sizeof(double) * tot, &d);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(d, f, sizeof(double) * tot, hipMemcpyHostToDevice, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        rc = store_populations(d);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(st()));
        steps = 0;
        refreshed_at_ = -1;
        surr_ok_ = false;
        have_delta_ = false;
        return HSLB_OK;
    }

    // Raw checkpoint: header, populations in storage precision [19][N], the
    // reference table [nz][19].
    struct CkHeader {
        int64_t magic, tf_bytes, nx, ny, nz, steps, refreshed_at, q;
    };
    static constexpr int64_t kMagic = 0x48534c4243503031;  // "HSLBCP01"

    int checkpoint_bytes(int64_t *bytes) override
    {
        *bytes = (int64_t)sizeof(CkHeader) + (int64_t)sizeof(TF) * q_ * L_.N + (int64_t)sizeof(double) * NQ * L_.nz;
        return HSLB_OK;
    }

    int checkpoint_save(void *buf) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "checkpoint before init");
        CkHeader h{kMagic, (int64_t)sizeof(TF), L_.nx, L_.ny, L_.nz, steps, refreshed_at_, q_};
        char *p = (char *)buf;
        std::memcpy(p, &h, sizeof(h));
        p += sizeof(h);
        for (int i = 0; i < q_; ++i) {
            HIP_TRY(hipMemcpyAsync(p, f_[cur_] + (size_t)i * L_.pop_stride, sizeof(TF) * L_.N, hipMemcpyDeviceToHost,
                                   st()));
            p += sizeof(TF) * L_.N;
        }
        HIP_TRY(hipMemcpyAsync(p, nref_d_, sizeof(double) * NQ * L_.nz, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int checkpoint_load(const void *buf) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "initialise before loading a checkpoint");
        CkHeader h;
        std::memcpy(&h, buf, sizeof(h));
        if (h.magic != kMagic || h.tf_bytes != (int64_t)sizeof(TF) || h.nx != L_.nx || h.ny != L_.ny ||
            h.nz != L_.nz || h.q != q_)
            return fail(err, HSLB_EINVAL, "checkpoint does not match this context");
        const char *p = (const char *)buf + sizeof(h);
        for (int i = 0; i < q_; ++i) {
            HIP_TRY(hipMemcpyAsync(f_[cur_] + (size_t)i * L_.pop_stride, p, sizeof(TF) * L_.N, hipMemcpyHostToDevice,
                                   st()));
            p += sizeof(TF) * L_.N;
        }
        HIP_TRY(hipMemcpyAsync(nref_d_, p, sizeof(double) * NQ * L_.nz, hipMemcpyHostToDevice, st()));
        HIP_TRY(hipMemcpyAsync(nref_d_ + NQ * L_.nz, p, sizeof(double) * NQ * L_.nz, hipMemcpyHostToDevice, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        steps = h.steps;
        refreshed_at_ = h.refreshed_at;
        surr_ok_ = false;
        have_delta_ = false;
        return HSLB_OK;
    }

    // ------------------------------------------------ learned force

    cnn::Geo cnn_geo() const { return cnn::Geo{L_.nx, L_.ny, L_.nz, L_.zper, L_.N}; }

    // Network buffers, allocated with the first weights.
    int surr_alloc()
    {
        if (surr_mem_) return HSLB_OK;
        const size_t N = L_.N;
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off += (bytes + 255) / 256 * 256;
            return o;
        };
        const size_t o_w = take(sizeof(float) * cnn::NW);
        size_t o_pk[3];
        for (int k = 0; k < 3; ++k) o_pk[k] = take(sizeof(uint16_t) * cnn::pack_elems(k));
        const size_t o_x = take(sizeof(uint16_t) * N);
        const size_t o_a1 = take(sizeof(uint16_t) * 32 * N);
        const size_t o_a2 = take(sizeof(uint16_t) * 32 * N);
        const size_t o_fh = take(sizeof(float) * 3 * N);
        const size_t o_dl = take(sizeof(float) * 3 * N);
        const size_t o_c1 = take(sizeof(double) * 3 * N);
        const size_t o_jp = take(sizeof(double) * 2 * cnn::judge_blocks(cnn_geo()));
        if (hipMalloc(&surr_mem_, off) != hipSuccess) return fail(err, HSLB_ENOMEM, "learned-force buffers (%zu bytes)", off);
        char *b = (char *)surr_mem_;
        cw_ = (float *)(b + o_w);
        for (int k = 0; k < 3; ++k) cpk_[k] = (uint16_t *)(b + o_pk[k]);
        cx_ = (uint16_t *)(b + o_x);
        ca1_ = (uint16_t *)(b + o_a1);
        ca2_ = (uint16_t *)(b + o_a2);
        fhat_ = (float *)(b + o_fh);
        delta_ = (float *)(b + o_dl);
        c1_ = (double *)(b + o_c1);
        jpart_ = (double *)(b + o_jp);
        HIP_TRY(hipMemset(delta_, 0, sizeof(float) * 3 * N));
        HIP_TRY(hipHostMalloc((void **)&jpart_h_, sizeof(double) * 2 * cnn::judge_blocks(cnn_geo()), hipHostMallocDefault));
        fscale_ = (1.0 / 3.0) * (6.0 / M_PI) * (6.0 / M_PI) * 4.0 * M_PI / std::pow((double)sigma_, 4);
        return HSLB_OK;
    }

    int surr_set_weights(const float *w) override
    {
        if (p_.force_mode != HSLB_FORCE_SURROGATE) return fail(err, HSLB_ESTATE, "context is not in surrogate mode");
        for (int i = 0; i < cnn::NW; ++i)
            if (!std::isfinite(w[i])) return fail(err, HSLB_EINVAL, "weight %d is not finite", i);
        int rc = surr_alloc();
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(cw_, w, sizeof(float) * cnn::NW, hipMemcpyHostToDevice, st()));
        for (int k = 0; k < 3; ++k) HIP_TRY(cnn::launch_pack(st(), k, cw_, cpk_[k]));
        HIP_TRY(hipStreamSynchronize(st()));
        have_w_ = true;
        surr_ok_ = false;
        have_delta_ = false;
        surr_checks_ = surr_fallback_ = 0;
        surr_last_r_ = -1.0;
        surr_max_r_ = 0.0;
        return HSLB_OK;
    }

    int surr_get_weights(float *w) override
    {
        if (!have_w_) return fail(err, HSLB_ENOSURR, "no weights loaded");
        HIP_TRY(hipMemcpyAsync(w, cw_, sizeof(float) * cnn::NW, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int surr_set_mode(int mode) override
    {
        if (p_.force_mode != HSLB_FORCE_SURROGATE) return fail(err, HSLB_ESTATE, "context is not in surrogate mode");
        if (mode < HSLB_SURR_CORRECTED || mode > HSLB_SURR_FROZEN) return fail(err, HSLB_EINVAL, "surrogate mode");
        surr_mode_ = mode;
        surr_ok_ = false;
        have_delta_ = false;
        return HSLB_OK;
    }

    int surr_set_components(int mask) override
    {
        if (p_.force_mode != HSLB_FORCE_SURROGATE) return fail(err, HSLB_ESTATE, "context is not in surrogate mode");
        if (mask < 1 || mask > 7) return fail(err, HSLB_EINVAL, "network force components: a mask of bits 0..2, not 0");
        surr_zero_ = ~mask & 7;
        surr_ok_ = false;
        have_delta_ = false;
        return HSLB_OK;
    }

    int surr_stats(int64_t *checks, int64_t *fallback, double *last_r, double *max_r) override
    {
        if (checks) *checks = surr_checks_;
        if (fallback) *fallback = surr_fallback_;
        if (last_r) *last_r = surr_last_r_;
        if (max_r) *max_r = surr_max_r_;
        return HSLB_OK;
    }

    // F_hat of the current moments (in fld_.n) into fhat_.
    int cnn_forward()
    {
        const cnn::Geo g = cnn_geo();
        const double eta_in = M_PI * std::pow((double)sigma_, 3) / 6.0;
        int rc = launch("cnn_input", [&] { return cnn::launch_eta_input<TM>(st(), g, L_.hz, eta_in, fld_.n, cx_); });
        if (rc) return rc;
        cnn::FwdArgs a{};
        a.g = g;
        a.in = cx_;
        a.wp = cpk_[0];
        a.bias = cw_ + cnn::OB1;
        a.out_cl = ca1_;
        if ((rc = launch("cnn_l1", [&] { return cnn::launch_conv_fwd(st(), 1, 32, cnn::EPI_GELU, a); }))) return rc;
        a.in = ca1_;
        a.wp = cpk_[1];
        a.bias = cw_ + cnn::OB2;
        a.out_cl = ca2_;
        if ((rc = launch("cnn_l2", [&] { return cnn::launch_conv_fwd(st(), 32, 32, cnn::EPI_GELU, a); }))) return rc;
        a.in = ca2_;
        a.wp = cpk_[2];
        a.bias = cw_ + cnn::OB3;
        a.out_cl = nullptr;
        a.out_f32 = fhat_;
        a.out_zero = surr_zero_;
        return launch("cnn_l3", [&] { return cnn::launch_conv_fwd(st(), 32, 3, cnn::EPI_OUT, a); });
    }

    // A step with the learned force (plus the frozen correction).
    int step_surrogate()
    {
        int rc = launch("moments", [&] { return launch_moments<TF, TM>(st(), L_, nref_d_, f_[cur_], fld_); });
        if (rc) return rc;
        if (surr_mode_ != HSLB_SURR_FROZEN && (rc = cnn_forward())) return rc;
        StepConst sc = sc_;
        sc.fext = surr_mode_ != HSLB_SURR_FROZEN ? fhat_ : nullptr;
        sc.fdelta = surr_mode_ != HSLB_SURR_PLAIN ? delta_ : nullptr;
        sc.fscale = fscale_;
        rc = launch("collide_ext", [&] {
            return launch_collide<TF, TM>(st(), L_, 0, sc, chi_d_, f_[cur_], f_[1 - cur_], fld_);
        });
        if (rc) return rc;
        cur_ = 1 - cur_;
        return HSLB_OK;
    }

    // Exact step that also judges the learned force: residual
    // |fs F_hat - C1| / |C1| over fluid nodes, correction C1 - fs F_hat.
    int step_check()
    {
        int rc = launch("moments", [&] { return launch_moments<TF, TM>(st(), L_, nref_d_, f_[cur_], fld_); });
        if (rc) return rc;
        if ((rc = fields_hs())) return rc;
        StepConst s0 = sc_;
        s0.g[0] = s0.g[1] = s0.g[2] = 0.0;
        if ((rc = launch("exact_c1", [&] {
                 return launch_force<TF, TM>(st(), L_, sigma_, s0, chi_d_, f_[cur_], fld_, c1_);
             })))
            return rc;
        const bool net = surr_mode_ != HSLB_SURR_FROZEN;
        if (net && (rc = cnn_forward())) return rc;
        // judge the force the path would apply now: with the correction of the
        // previous check (corrected and frozen modes), the bare network (plain)
        const int use_prev = have_delta_ && surr_mode_ != HSLB_SURR_PLAIN ? 1 : 0;
        const cnn::Geo g = cnn_geo();
        const unsigned nb = cnn::judge_blocks(g);
        if ((rc = launch("judge", [&] {
                 return cnn::launch_judge(st(), g, L_.zper ? 0 : L_.wall_lo, L_.zper ? 0 : L_.wall_hi, net ? fscale_ : 0.0,
                                          net ? fhat_ : nullptr, c1_, use_prev, delta_, jpart_);
             })))
            return rc;
        HIP_TRY(hipMemcpyAsync(jpart_h_, jpart_, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st()));
        rc = launch("collide", [&] {
            return launch_collide<TF, TM>(st(), L_, sigma_, sc_, chi_d_, f_[cur_], f_[1 - cur_], fld_, collide_tiles);
        });
        if (rc) return rc;
        cur_ = 1 - cur_;
        HIP_TRY(hipStreamSynchronize(st()));
        double a = 0.0, b = 0.0;
        for (unsigned k = 0; k < nb; ++k) {
            a += jpart_h_[2 * k];
            b += jpart_h_[2 * k + 1];
        }
        // a non-finite state or force fails the check
        const double r = !(std::isfinite(a) && std::isfinite(b)) ? INFINITY
                         : b > 0.0                                ? std::sqrt(a / b)
                         : a > 0.0                                ? INFINITY
                                                                  : 0.0;
        surr_last_r_ = r;
        surr_max_r_ = std::max(surr_max_r_, r);
        surr_checks_ += 1;
        have_delta_ = true;
        surr_ok_ = r <= p_.surr_tol;
        return HSLB_OK;
    }

    int advance_surrogate(int64_t n)
    {
        if (!have_w_) return fail(err, HSLB_ENOSURR, "no surrogate weights loaded");
        const int64_t K = p_.surr_check_every;
        while (n > 0) {
            const bool refresh =
                shift_every > 0 && steps > 0 && steps % shift_every == 0 && refreshed_at_ != steps;
            if (refresh)
                HIP_TRY(launch_layer_means<TF>(st(), L_, f_[cur_], L_.pop_stride, nref_d_, nref_d_ + NQ * L_.nz));
            int rc;
            if (steps % K == 0 || !surr_ok_) {
                if (steps % K == 0) {
                    rc = step_check();
                } else {
                    surr_fallback_ += 1;
                    rc = one_step();
                }
            } else {
                rc = step_surrogate();
            }
            if (rc) return rc;
            if (refresh) {
                HIP_TRY(hipMemcpyAsync(nref_d_, nref_d_ + NQ * L_.nz, sizeof(double) * NQ * L_.nz,
                                       hipMemcpyDeviceToDevice, st()));
                refreshed_at_ = steps;
            }
            n -= 1;
            steps += 1;
        }
        return HSLB_OK;
    }

    int surr_force(double *F) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "force before init");
        if (!have_w_) return fail(err, HSLB_ENOSURR, "no surrogate weights loaded");
        double *d;
        const size_t N = L_.N;
        int rc = io(sizeof(double) * 3 * N, &d);
        if (rc) return rc;
        HIP_TRY(launch_moments<TF, TM>(st(), L_, nref_d_, f_[cur_], fld_));
        if ((rc = cnn_forward())) return rc;
        HIP_TRY(cnn::launch_scale_f32_to_f64(st(), fhat_, fscale_, 3 * N, d));
        HIP_TRY(hipMemcpyAsync(F, d, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int training_pair(uint16_t *x, float *target, cnn::Geo *g, int *wall_lo, int *wall_hi, int *sigma) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "snapshot before init");
        if (p_.force_mode == HSLB_FORCE_OFF) return fail(err, HSLB_ESTATE, "hard-sphere term is off");
        if (l39()) return fail(err, HSLB_EINVAL, "training snapshots come from 19-velocity lattices");
        if (L_.nx % 32 || L_.ny % 4) return fail(err, HSLB_EINVAL, "training snapshots need nx %% 32 == 0 and ny %% 4 == 0");
        if (!x || !target) {  // geometry only
            *g = cnn_geo();
            *wall_lo = L_.zper ? 0 : L_.wall_lo;
            *wall_hi = L_.zper ? 0 : L_.wall_hi;
            *sigma = sigma_;
            return HSLB_OK;
        }
        double *d;
        const size_t N = L_.N;
        int rc = io(sizeof(double) * 3 * N, &d);
        if (rc) return rc;
        const double fs = (1.0 / 3.0) * (6.0 / M_PI) * (6.0 / M_PI) * 4.0 * M_PI / std::pow((double)sigma_, 4);
        HIP_TRY(launch_moments<TF, TM>(st(), L_, nref_d_, f_[cur_], fld_));
        if ((rc = fields_hs())) return rc;
        StepConst s0 = sc_;
        s0.g[0] = s0.g[1] = s0.g[2] = 0.0;
        HIP_TRY(launch_force<TF, TM>(st(), L_, sigma_, s0, chi_d_, f_[cur_], fld_, d));
        HIP_TRY(cnn::launch_scale_f64_to_f32(st(), d, 1.0 / fs, 3 * N, target));
        HIP_TRY(cnn::launch_eta_input<TM>(st(), cnn_geo(), L_.hz, M_PI * std::pow((double)sigma_, 3) / 6.0, fld_.n, x));
        HIP_TRY(hipStreamSynchronize(st()));
        *g = cnn_geo();
        *wall_lo = L_.zper ? 0 : L_.wall_lo;
        *wall_hi = L_.zper ? 0 : L_.wall_hi;
        *sigma = sigma_;
        return HSLB_OK;
    }

private:
    // learned force
    void *surr_mem_ = nullptr;
    float *cw_ = nullptr;
    uint16_t *cpk_[3] = {nullptr, nullptr, nullptr};
    uint16_t *cx_ = nullptr, *ca1_ = nullptr, *ca2_ = nullptr;
    float *fhat_ = nullptr, *delta_ = nullptr;
    double *c1_ = nullptr, *jpart_ = nullptr, *jpart_h_ = nullptr;
    double fscale_ = 0.0;
    bool have_w_ = false, surr_ok_ = false, have_delta_ = false;
    int surr_mode_ = HSLB_SURR_CORRECTED;
    int surr_zero_ = 0;  // network force components (bit c) held at 0
    int64_t surr_checks_ = 0, surr_fallback_ = 0;
    double surr_last_r_ = -1.0, surr_max_r_ = 0.0;

    hslb_params p_;
    LatticeDev L_{};
    StepConst sc_{};
    AttWeights aw_{};
    double *att_d_ = nullptr;  // attraction: x-pass, y-pass, potential [N] each
    std::vector<uint8_t> solid_h_;  // solid mask (empty: walls only)
    uint32_t *links_d_ = nullptr;   // [N] solid-neighbour bits (mask set)
    double *chi_n_d_ = nullptr;     // [N] per-node wall factor (mask set)
    int sigma_ = 2;
    int q_ = NQ;  // velocities: 19, or 39 for the third-order lattice (FP64)
    bool thermal_ = false;  // non-isothermal terms (39 velocities)
    bool l39() const { return q_ == Q39; }
    hipStream_t stream_ = nullptr, ext_stream_ = nullptr;
    bool own_stream_ = false;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    TF *f_[2] = {nullptr, nullptr};
    int cur_ = 0;
    TM *fld_mem_ = nullptr;
    TM *rs_ = nullptr;
    Fields<TM> fld_{};
    double *chi_d_ = nullptr, *prof_d_ = nullptr, *prof_h_ = nullptr;
    double *nref_d_ = nullptr;  // [2][nz][19]: read table, write table
    double *io_d_ = nullptr;
    size_t io_bytes_ = 0;
    double mass0_ = 0.0;
    int64_t last_steps_ = 0;
    hipGraphExec_t gexecL_[2] = {nullptr, nullptr};  // HSLB_GRAPH_LONG steps per replay
    hipGraphExec_t gexec_[2] = {nullptr, nullptr};
    bool capturing_ = false;
    int64_t refreshed_at_ = -1;
};

// ------------------------------------------------------------------ batch

// Per-slit constants, built on the host exactly as for a single lattice.
void slit_consts(const hslb_params &p, LatticeDev &L, StepConst &sc, std::vector<double> &chi)
{
    const int sig = p.sigma >= 2 ? p.sigma : 2;
    L.nx = p.nx;
    L.ny = p.ny;
    L.nz = p.nz;
    L.wall_lo = p.wall_lo;
    L.wall_hi = p.wall_hi;
    L.zper = (p.wall_lo == 0 && p.wall_hi == 0) ? 1 : 0;
    L.hz = sig;
    L.plane = p.nx * p.ny;
    L.N = L.plane * p.nz;
    sc.tau = p.tau;
    for (int a = 0; a < 3; ++a) sc.g[a] = p.accel[a];
    const double vt2 = 1.0 / 3.0;
    sc.pref = -vt2 * (double)sig * (double)sig * 4.0 * M_PI;
    sc.kappa = 2.0 / (std::sqrt(vt2) * std::sqrt(M_PI));
    sc.eta_pref = M_PI * (double)sig * sig * sig / 6.0 / (double)ball_count(sig);
    const double A = (double)sig / std::sqrt(2.0);
    const double th = A - std::floor(A);
    sc.alpha[0] = (1.0 - th) * (1.0 - th);
    sc.alpha[1] = (1.0 - th) * th;
    sc.alpha[2] = th * (1.0 - th);
    sc.alpha[3] = th * th;
    sc.g2_model = p.g2_model;
    sc.hs_on = (p.force_mode == HSLB_FORCE_OFF) ? 0 : 1;
    sc.phi = nullptr;
    sc.links = nullptr;
    sc.chi_n = nullptr;
    chi.assign(p.nz, 1.0);
    if (!L.zper && p.wall_reg) {
        const double za = p.wall_lo - 0.5, zb = p.nz - p.wall_hi - 0.5;
        for (int z = 0; z < p.nz; ++z) chi[z] = 1.0 - std::exp(-std::fmin((double)z - za, zb - (double)z) / (double)sig);
    }
}

// A ragged ensemble of independent slits advanced together: five persistent
// launches per step (moments, row sums, ball sums, contact values, collide)
// over work lists that span every slit, K steps per captured HIP graph.
template <typename TF, typename TM>
class BatchT final : public Engine {
public:
    explicit BatchT(std::vector<hslb_params> p) : p_(std::move(p)) {}

    ~BatchT() override
    {
        drop_graphs();
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
        (void)hipFree(f_[0]);
        (void)hipFree(f_[1]);
        (void)hipFree(fld_mem_);
        (void)hipFree(aux_);
        (void)hipHostFree(prof_h_);
        (void)hipFree(io_d_);
        if (stream_) (void)hipStreamDestroy(stream_);
    }

    int setup()
    {
        const int ns = (int)p_.size();
        desc_.resize(ns);
        std::vector<double> chi_all;
        int64_t pop = 0, fld = 0, prof = 0;
        int maxR = 0;
        rows16_ = ns > 0;
        fused_rows_ = ns > 0;
        for (int k = 0; k < ns; ++k) {
            SlitDesc &d = desc_[k];
            std::vector<double> chi;
            slit_consts(p_[k], d.L, d.sc, chi);
            rows16_ = rows16_ && d.L.nx == 16;
            fused_rows_ = fused_rows_ && 256 % d.L.nx == 0 && d.L.plane % 256 == 0;
            d.sigma = p_[k].sigma >= 2 ? p_[k].sigma : 2;
            maxR = std::max(maxR, d.sigma / 2);
            d.pop_off = (int)pop;
            d.fld_off = (int)fld;
            d.chi_off = (int)chi_all.size();
            chi_all.insert(chi_all.end(), chi.begin(), chi.end());
            pop += (d.L.N + 63) / 64 * 64;
            fld += ((int64_t)d.L.plane * (d.L.nz + 2 * d.L.hz) + 63) / 64 * 64;
            prof_off_.push_back((int)prof);
            prof += 5 * (int64_t)d.L.nz;
            nfluid_ += (int64_t)d.L.plane * (d.L.nz - d.L.wall_lo - d.L.wall_hi);
        }
        if (pop * NQ >= ((int64_t)1 << 31) || fld * 8 >= ((int64_t)1 << 31))
            return fail(err, HSLB_EINVAL, "ensemble too large for 32-bit indices");
        pop_stride_ = (int)pop;
        fld_stride_ = (int)((fld + 63) / 64 * 64);
        for (auto &d : desc_) {
            d.L.pop_stride = pop_stride_;
            d.L.fld_stride = fld_stride_;
        }
        nprof_ = (int)prof;
        // work lists: all nodes, row-sum rows, fluid nodes; profile items (slit, z)
        for (int k = 0; k < ns; ++k) {
            const LatticeDev &L = desc_[k].L;
            const int R = desc_[k].sigma / 2;
            const int nfl = L.zper ? L.N : (L.nz - L.wall_lo - L.wall_hi) * L.plane;
            for (int b = 0; b < (L.N + 255) / 256; ++b) wl_nodes_.push_back({k, b});
            for (int b = 0; b < (L.plane * (L.nz + 2 * R) + 255) / 256; ++b) wl_rows_.push_back({k, b});
            for (int b = 0; b < (nfl + 255) / 256; ++b) wl_fluid_.push_back({k, b});
            for (int z = 0; z < L.nz; ++z) wl_prof_.push_back({k, z});
        }
        HIP_TRY(hipStreamCreate(&stream_));
        HIP_TRY(hipEventCreate(&ev0_));
        HIP_TRY(hipEventCreate(&ev1_));
        const size_t popb = sizeof(TF) * (size_t)NQ * pop_stride_;
        if (hipMalloc(&f_[0], popb) != hipSuccess || hipMalloc(&f_[1], popb) != hipSuccess)
            return fail(err, HSLB_ENOMEM, "population buffers (%zu bytes each) do not fit", popb);
        HIP_TRY(hipMemset(f_[0], 0, popb));
        HIP_TRY(hipMemset(f_[1], 0, popb));
        const size_t nf = (size_t)(1 + 4 + 1 + NGSLOT + maxR + 1) * fld_stride_;
        if (hipMalloc(&fld_mem_, sizeof(TM) * nf) != hipSuccess) return fail(err, HSLB_ENOMEM, "moment fields");
        HIP_TRY(hipMemset(fld_mem_, 0, sizeof(TM) * nf));
        fld_.n = fld_mem_;
        fld_.nj = fld_mem_ + fld_stride_;
        fld_.eb = fld_mem_ + 5 * (size_t)fld_stride_;
        fld_.G = fld_mem_ + 6 * (size_t)fld_stride_;
        rs_ = fld_mem_ + (size_t)(6 + NGSLOT) * fld_stride_;
        // descriptors, work lists, chi, profile offsets and profiles in one block
        const size_t bdesc = sizeof(SlitDesc) * ns;
        const size_t bw = sizeof(WorkItem) * (wl_nodes_.size() + wl_rows_.size() + wl_fluid_.size() + wl_prof_.size());
        const size_t bchi = sizeof(double) * chi_all.size();
        const size_t bpo = sizeof(int) * ns;
        const size_t bprof = sizeof(double) * nprof_;
        const size_t bref = sizeof(double) * 2 * NQ * chi_all.size();
        auto al = [](size_t b) { return (b + 255) / 256 * 256; };
        HIP_TRY(hipMalloc(&aux_, al(bdesc) + al(bw) + al(bchi) + al(bpo) + al(bprof) + al(bref)));
        char *a = (char *)aux_;
        desc_d_ = (SlitDesc *)a;
        a += al(bdesc);
        work_d_ = (WorkItem *)a;
        a += al(bw);
        chi_d_ = (double *)a;
        a += al(bchi);
        prof_off_d_ = (int *)a;
        a += al(bpo);
        prof_d_ = (double *)a;
        a += al(bprof);
        nref_d_ = (double *)a;
        ztot_ = (int)chi_all.size();
        HIP_TRY(hipMemset(nref_d_, 0, bref));
        for (auto &d : desc_) {
            d.sc.nref_r = nref_d_ + (size_t)NQ * d.chi_off;
            d.sc.nref_w = nref_d_ + (size_t)NQ * (ztot_ + d.chi_off);
        }
        shift_every = (sizeof(TF) == 4) ? 50 : 0;
        HIP_TRY(hipMemcpy(desc_d_, desc_.data(), bdesc, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(chi_d_, chi_all.data(), bchi, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(prof_off_d_, prof_off_.data(), bpo, hipMemcpyHostToDevice));
        HIP_TRY(upload_work(0));
        HIP_TRY(hipHostMalloc((void **)&prof_h_, bprof, hipHostMallocDefault));
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&ncu_, hipDeviceAttributeMultiprocessorCount, dev));
        inited_.assign(ns, 0);
        return HSLB_OK;
    }

    // Order 0: slit order; 1: grouped by sigma (largest stencils first).
    hipError_t upload_work(int order)
    {
        auto sorted = [&](std::vector<WorkItem> v) {
            if (order == 1)
                std::stable_sort(v.begin(), v.end(), [&](const WorkItem &a, const WorkItem &b) {
                    return desc_[a.slit].sigma > desc_[b.slit].sigma;
                });
            return v;
        };
        std::vector<WorkItem> all;
        for (auto *wl : {&wl_nodes_, &wl_rows_, &wl_fluid_}) {
            auto v = sorted(*wl);
            all.insert(all.end(), v.begin(), v.end());
        }
        all.insert(all.end(), wl_prof_.begin(), wl_prof_.end());
        order_ = order;
        return hipMemcpy(work_d_, all.data(), sizeof(WorkItem) * all.size(), hipMemcpyHostToDevice);
    }

    void set_stream(hipStream_t s) override { ext_stream_ = s; }
    hipStream_t st() const { return ext_stream_ ? ext_stream_ : stream_; }

    void drop_graphs()
    {
        for (auto &g : gexec_)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }

    int io(size_t bytes, double **out)
    {
        if (bytes > io_bytes_) {
            (void)hipFree(io_d_);
            io_d_ = nullptr;
            io_bytes_ = 0;
            if (hipMalloc(&io_d_, bytes) != hipSuccess) return fail(err, HSLB_ENOMEM, "staging buffer");
            io_bytes_ = bytes;
        }
        *out = io_d_;
        return HSLB_OK;
    }

    int batch_init(int slit, const double *n, const double *u) override
    {
        if (slit < 0 || slit >= (int)p_.size()) return fail(err, HSLB_EINVAL, "slit %d out of range", slit);
        SlitDesc &d = desc_[slit];
        const int N = d.L.N;
        double msum = 0.0;
        int64_t nfl = 0;
        for (int id = 0; id < N; ++id) {
            const int z = id / d.L.plane;
            if (!(d.L.zper || (z >= d.L.wall_lo && z < d.L.nz - d.L.wall_hi))) continue;
            if (!std::isfinite(n[id]) || n[id] < 0.0)
                return fail(err, HSLB_EINVAL, "slit %d: density at node %d is negative or not finite", slit, id);
            if (u)
                for (int a = 0; a < 3; ++a)
                    if (!std::isfinite(u[(size_t)a * N + id]))
                        return fail(err, HSLB_EINVAL, "slit %d: velocity at node %d is not finite", slit, id);
            msum += n[id];
            ++nfl;
        }
        double *dd;
        int rc = io(sizeof(double) * (4 + NQ) * (size_t)N, &dd);
        if (rc) return rc;
        double *stage = dd + 4 * (size_t)N;
        HIP_TRY(hipMemcpyAsync(dd, n, sizeof(double) * N, hipMemcpyHostToDevice, st()));
        if (u)
            HIP_TRY(hipMemcpyAsync(dd + N, u, sizeof(double) * 3 * (size_t)N, hipMemcpyHostToDevice, st()));
        else
            HIP_TRY(hipMemsetAsync(dd + N, 0, sizeof(double) * 3 * (size_t)N, st()));
        HIP_TRY(launch_feq(st(), d.L, dd, dd + N, stage));
        double *R = nref_d_ + (size_t)NQ * d.chi_off, *W = nref_d_ + (size_t)NQ * (ztot_ + d.chi_off);
        HIP_TRY(launch_layer_means<double>(st(), d.L, stage, N, nullptr, R));
        HIP_TRY(hipMemcpyAsync(W, R, sizeof(double) * NQ * d.L.nz, hipMemcpyDeviceToDevice, st()));
        HIP_TRY(launch_set_pop<TF>(st(), d.L, R, stage, f_[cur_] + d.pop_off));
        HIP_TRY(hipStreamSynchronize(st()));
        inited_[slit] = 1;
        steps = 0;
        refreshed_at_ = -1;
        inited = std::all_of(inited_.begin(), inited_.end(), [](char c) { return c != 0; });
        return HSLB_OK;
    }

    int init(const double *, const double *) override { return fail_state("use hslb_batch_init on a batch"); }

    int phase(const char *name, int ph, const WorkItem *w, int nw)
    {
        hipEvent_t a = nullptr, b = nullptr;
        if (kt.enabled && !capturing_) {
            HIP_TRY(kt.ev(&a));
            HIP_TRY(kt.ev(&b));
            HIP_TRY(hipEventRecord(a, st()));
        }
        const unsigned grid = (unsigned)std::max(1, std::min(nw, ncu_ * grid_per_cu_));
        HIP_TRY(launch_batch_phase<TF, TM>(st(), ph, grid, desc_d_, w, nw, f_[cur_], f_[1 - cur_], fld_, rs_, chi_d_,
                                           rows16_));
        if (a) {
            HIP_TRY(hipEventRecord(b, st()));
            kt.pending.push_back({name, {(int)kt.used - 2, (int)kt.used - 1}});
        }
        return HSLB_OK;
    }

    int collide(const WorkItem *wf, int nw)
    {
        hipEvent_t a = nullptr, b = nullptr;
        if (kt.enabled && !capturing_) {
            HIP_TRY(kt.ev(&a));
            HIP_TRY(kt.ev(&b));
            HIP_TRY(hipEventRecord(a, st()));
        }
        const unsigned grid = (unsigned)std::max(1, std::min(nw, ncu_ * cgrid_per_cu_));
        HIP_TRY(launch_batch_collide<TF, TM>(st(), grid, desc_d_, wf, nw, f_[cur_], f_[1 - cur_], fld_, chi_d_,
                                             rows16_));
        if (a) {
            HIP_TRY(hipEventRecord(b, st()));
            kt.pending.push_back({"b_collide", {(int)kt.used - 2, (int)kt.used - 1}});
        }
        return HSLB_OK;
    }

    int one_step()
    {
        const WorkItem *wn = work_d_, *wr = wn + wl_nodes_.size(), *wf = wr + wl_rows_.size();
        int rc;
        if (fused_rows_) {
            // 512 16x16 slits: 90 + 41 -> 100 us (moments and row sums)
            if ((rc = phase("b_moments", 4, wn, (int)wl_nodes_.size()))) return rc;
        } else {
            if ((rc = phase("b_moments", 0, wn, (int)wl_nodes_.size()))) return rc;
            if ((rc = phase("b_rowsum", 1, wr, (int)wl_rows_.size()))) return rc;
        }
        if ((rc = phase("b_ballsum", 2, wn, (int)wl_nodes_.size()))) return rc;
        if ((rc = phase("b_gfield", 3, wn, (int)wl_nodes_.size()))) return rc;
        if ((rc = collide(wf, (int)wl_fluid_.size()))) return rc;
        cur_ = 1 - cur_;
        return HSLB_OK;
    }

    int capture(int parity)
    {
        const int save = cur_;
        cur_ = parity;
        capturing_ = true;
        HIP_TRY(hipStreamBeginCapture(st(), hipStreamCaptureModeThreadLocal));
        int rc = HSLB_OK;
        for (int k = 0; k < graph_steps_ && !rc; ++k) rc = one_step();
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st(), &g);
        capturing_ = false;
        cur_ = save;
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(err, HSLB_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&gexec_[parity], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(err, HSLB_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
        return HSLB_OK;
    }

    int prepare() override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "prepare before every slit is initialised");
        if (!use_graph || kt.enabled) return HSLB_OK;
        for (int par = 0; par < 2; ++par) {
            if (!gexec_[par]) {
                int rc = capture(par);
                if (rc) return rc;
            }
        }
        return HSLB_OK;
    }

    int refresh_step()
    {
        const WorkItem *wp = work_d_ + wl_nodes_.size() + wl_rows_.size() + wl_fluid_.size();
        HIP_TRY(launch_batch_layer_means<TF>(st(), desc_d_, wp, (int)wl_prof_.size(), f_[cur_]));
        int rc = one_step();
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(nref_d_, nref_d_ + (size_t)NQ * ztot_, sizeof(double) * NQ * ztot_,
                               hipMemcpyDeviceToDevice, st()));
        return HSLB_OK;
    }

    int advance(int64_t n)
    {
        const bool graph = use_graph && !kt.enabled;
        while (n > 0) {
            if (shift_every > 0 && steps > 0 && steps % shift_every == 0 && refreshed_at_ != steps) {
                int rc = refresh_step();
                if (rc) return rc;
                refreshed_at_ = steps;
                n -= 1;
                steps += 1;
                continue;
            }
            const int64_t room = shift_every > 0 ? shift_every - steps % shift_every : n;
            if (graph && n >= graph_steps_ && room >= graph_steps_) {
                if (!gexec_[cur_]) {
                    int rc = capture(cur_);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(gexec_[cur_], st()));
                n -= graph_steps_;
                steps += graph_steps_;
                if (graph_steps_ % 2) cur_ = 1 - cur_;
            } else {
                int rc = one_step();
                if (rc) return rc;
                n -= 1;
                steps += 1;
            }
        }
        return HSLB_OK;
    }

    int step(int64_t nsteps) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "step before every slit is initialised");
        if (nsteps < 0) return fail(err, HSLB_EINVAL, "negative step count");
        HIP_TRY(hipEventRecord(ev0_, st()));
        int rc = advance(nsteps);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ev1_, st()));
        last_steps_ = nsteps;
        prof_valid_ = false;
        if (kt.enabled && !kt.pending.empty()) {
            HIP_TRY(hipStreamSynchronize(st()));
            for (auto &pr : kt.pending) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, kt.pool[pr.second.first], kt.pool[pr.second.second]));
                auto &t = kt.totals[pr.first];
                t.first += ms;
                t.second += 1;
            }
            kt.pending.clear();
            kt.used = 0;
        }
        return HSLB_OK;
    }

    int sync() override
    {
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int timings(double *ms, double *mlups) override
    {
        HIP_TRY(hipEventSynchronize(ev1_));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, ev0_, ev1_));
        const double per = last_steps_ > 0 ? (double)t / (double)last_steps_ : 0.0;
        if (ms) *ms = per;
        if (mlups) *mlups = per > 0 ? (double)nfluid_ / (per * 1e-3) / 1e6 : 0.0;
        return HSLB_OK;
    }

    int refresh_profiles()
    {
        if (prof_valid_) return HSLB_OK;
        const WorkItem *wp = work_d_ + wl_nodes_.size() + wl_rows_.size() + wl_fluid_.size();
        HIP_TRY(launch_batch_profiles<TF>(st(), desc_d_, wp, (int)wl_prof_.size(), prof_off_d_, f_[cur_], prof_d_));
        HIP_TRY(hipMemcpyAsync(prof_h_, prof_d_, sizeof(double) * nprof_, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        prof_valid_ = true;
        return HSLB_OK;
    }

    int batch_profiles(int slit, double *nz, double *uz) override
    {
        if (slit < 0 || slit >= (int)p_.size()) return fail(err, HSLB_EINVAL, "slit %d out of range", slit);
        if (!inited) return fail(err, HSLB_ESTATE, "profiles before init");
        int rc = refresh_profiles();
        if (rc) return rc;
        const int n = desc_[slit].L.nz;
        const double *o = prof_h_ + prof_off_[slit];
        if (nz) std::memcpy(nz, o, sizeof(double) * n);
        if (uz) std::memcpy(uz, o + n, sizeof(double) * 3 * n);
        return HSLB_OK;
    }

    int batch_finite(int32_t *flags) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "finite check before init");
        int rc = refresh_profiles();
        if (rc) return rc;
        for (size_t k = 0; k < p_.size(); ++k) {
            const double *o = prof_h_ + prof_off_[k];
            bool ok = true;
            for (int i = 0; i < 5 * desc_[k].L.nz; ++i) ok = ok && std::isfinite(o[i]);
            flags[k] = ok ? 1 : 0;
        }
        return HSLB_OK;
    }

    int batch_set_config(int32_t grid_per_cu, int32_t order) override
    {
        return batch_set_launch(grid_per_cu, grid_per_cu, order);
    }

    int batch_set_launch(int32_t phase_grid, int32_t collide_grid, int32_t order) override
    {
        if (phase_grid < 1 || phase_grid > 1024 || collide_grid < 1 || collide_grid > 1024 || order < 0 || order > 1)
            return fail(err, HSLB_EINVAL, "batch launch configuration");
        grid_per_cu_ = phase_grid;
        cgrid_per_cu_ = collide_grid;
        if (order != order_) HIP_TRY(upload_work(order));
        drop_graphs();
        return HSLB_OK;
    }

    int batch_get_launch(int32_t *phase_grid, int32_t *collide_grid, int32_t *order) override
    {
        if (phase_grid) *phase_grid = grid_per_cu_;
        if (collide_grid) *collide_grid = cgrid_per_cu_;
        if (order) *order = order_;
        return HSLB_OK;
    }

    // Key of the tuning cache: device, storage precision and the slits'
    // geometry and sigma in order (FNV-1a 64).
    std::string tune_key() const
    {
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](int64_t v) {
            for (int k = 0; k < 8; ++k) {
                h ^= (uint64_t)((v >> (8 * k)) & 0xff);
                h *= 1099511628211ull;
            }
        };
        for (const auto &p : p_) {
            mix(p.nx), mix(p.ny), mix(p.nz), mix(p.wall_lo), mix(p.wall_hi), mix(p.sigma);
        }
        int dev = 0;
        hipDeviceProp_t prop{};
        std::string arch = "gpu";
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            arch = prop.gcnArchName;
            arch = arch.substr(0, arch.find(':'));
        }
        char buf[160];
        std::snprintf(buf, sizeof(buf), "hslb-batch-v1|%s|%s|%d|%016llx", arch.c_str(),
                      sizeof(TF) == 4 ? "f32" : "f64", (int)p_.size(), (unsigned long long)h);
        return buf;
    }

    // The cache file holds one JSON object; each line below its opening
    // brace is one entry "key": {"phase_grid": g, "collide_grid": c,
    // "order": o, "us_per_step": t}, as written by tune_store.
    static std::map<std::string, std::string> tune_read(const char *path)
    {
        std::map<std::string, std::string> out;
        FILE *f = std::fopen(path, "r");
        if (!f) return out;
        char line[1024];
        while (std::fgets(line, sizeof(line), f)) {
            const char *q0 = std::strchr(line, '"');
            const char *q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
            const char *br = q1 ? std::strchr(q1, '{') : nullptr;
            const char *be = br ? std::strchr(br, '}') : nullptr;
            if (!be) continue;
            out[std::string(q0 + 1, q1)] = std::string(br, be + 1);
        }
        std::fclose(f);
        return out;
    }

    static bool tune_parse(const std::string &v, int *pg, int *cg, int *order, double *us)
    {
        return std::sscanf(v.c_str(), "{\"phase_grid\": %d, \"collide_grid\": %d, \"order\": %d, \"us_per_step\": %lf}",
                           pg, cg, order, us) == 4;
    }

    static void tune_store(const char *path, const std::string &key, int pg, int cg, int order, double us)
    {
        auto all = tune_read(path);
        char v[256];
        std::snprintf(v, sizeof(v), "{\"phase_grid\": %d, \"collide_grid\": %d, \"order\": %d, \"us_per_step\": %.3f}",
                      pg, cg, order, us);
        all[key] = v;
        const std::string tmp = std::string(path) + ".tmp";
        FILE *f = std::fopen(tmp.c_str(), "w");
        if (!f) return;
        std::fprintf(f, "{\n");
        size_t k = 0;
        for (const auto &e : all)
            std::fprintf(f, "  \"%s\": %s%s\n", e.first.c_str(), e.second.c_str(), ++k < all.size() ? "," : "");
        std::fprintf(f, "}\n");
        const bool ok = std::fclose(f) == 0;
        if (ok) std::rename(tmp.c_str(), path);
    }

    // Time launch configurations over `nsteps` replayed steps each and keep
    // the fastest: (1) one grid for every phase, 1..32 blocks per compute
    // unit, slit order; (2) that phase grid with the other collide grids;
    // (3) the best of these with the work grouped by sigma.  The state is
    // saved before and restored after.  With HSLB_TUNE_CACHE naming a file,
    // a configuration stored there for the same device, precision and slits is
    // applied without timing (*choice = -1, us[0] = its stored time), and a
    // new result is added to the file.
    int batch_autotune(int32_t nsteps, int32_t *choice, double *us, int32_t cap) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "autotune before init");
        const char *cache = std::getenv("HSLB_TUNE_CACHE");
        const std::string key = tune_key();
        if (cache && *cache) {
            auto all = tune_read(cache);
            auto it = all.find(key);
            int pg, cg, order;
            double t;
            if (it != all.end() && tune_parse(it->second, &pg, &cg, &order, &t)) {
                int rc = batch_set_launch(pg, cg, order);
                if (rc) return rc;
                if (choice) *choice = -1;
                if (us && cap > 0) us[0] = t;
                return HSLB_OK;
            }
        }
        const int grids[] = {1, 2, 4, 8, 16, 32};
        const size_t popb = sizeof(TF) * (size_t)NQ * pop_stride_;
        TF *save = nullptr;
        if (hipMalloc(&save, popb) != hipSuccess) return fail(err, HSLB_ENOMEM, "autotune snapshot");
        HIP_TRY(hipMemcpyAsync(save, f_[cur_], popb, hipMemcpyDeviceToDevice, st()));
        std::vector<double> save_ref(2 * (size_t)NQ * ztot_);
        HIP_TRY(hipMemcpyAsync(save_ref.data(), nref_d_, sizeof(double) * save_ref.size(), hipMemcpyDeviceToHost,
                               st()));
        HIP_TRY(hipStreamSynchronize(st()));
        const int save_cur = cur_;
        const int64_t save_steps = steps, save_refreshed = refreshed_at_;
        struct Cand {
            int pg, cg, order;
            double us;
        };
        std::vector<Cand> cands;
        auto run = [&](int pg, int cg, int order) -> int {
            int rc = batch_set_launch(pg, cg, order);
            if (!rc) rc = advance(2);  // warm (and capture)
            if (!rc && hipEventRecord(ev0_, st()) != hipSuccess) rc = HSLB_EDEVICE;
            if (!rc) rc = advance(nsteps);
            float ms = 0.f;
            if (!rc && (hipEventRecord(ev1_, st()) != hipSuccess || hipEventSynchronize(ev1_) != hipSuccess ||
                        hipEventElapsedTime(&ms, ev0_, ev1_) != hipSuccess))
                rc = fail(err, HSLB_EDEVICE, "autotune timing");
            if (!rc) cands.push_back({pg, cg, order, 1e3 * ms / nsteps});
            return rc;
        };
        auto best_of = [&]() {
            size_t b = 0;
            for (size_t k = 1; k < cands.size(); ++k)
                if (cands[k].us < cands[b].us) b = k;
            return b;
        };
        int rc = HSLB_OK;
        for (int g : grids)
            if (!rc) rc = run(g, g, 0);
        const int pg = rc ? 8 : cands[best_of()].pg;
        for (int g : grids)
            if (!rc && g != pg) rc = run(pg, g, 0);
        if (!rc) {
            const Cand b = cands[best_of()];
            rc = run(b.pg, b.cg, 1);
        }
        if (rc) {
            (void)hipFree(save);
            return rc;
        }
        cur_ = save_cur;
        HIP_TRY(hipMemcpyAsync(f_[cur_], save, popb, hipMemcpyDeviceToDevice, st()));
        HIP_TRY(hipMemcpyAsync(nref_d_, save_ref.data(), sizeof(double) * save_ref.size(), hipMemcpyHostToDevice,
                               st()));
        HIP_TRY(hipStreamSynchronize(st()));
        (void)hipFree(save);
        steps = save_steps;
        refreshed_at_ = save_refreshed;
        prof_valid_ = false;
        const size_t best = best_of();
        for (size_t k = 0; k < cands.size() && us && (int32_t)k < cap; ++k) us[k] = cands[k].us;
        rc = batch_set_launch(cands[best].pg, cands[best].cg, cands[best].order);
        if (rc) return rc;
        if (choice) *choice = (int32_t)best;
        if (cache && *cache) tune_store(cache, key, cands[best].pg, cands[best].cg, cands[best].order, cands[best].us);
        return HSLB_OK;
    }

    int moments(double *, double *) override { return fail_state("use hslb_batch_profiles on a batch"); }
    int profiles(double *, double *) override { return fail_state("use hslb_batch_profiles on a batch"); }
    int force(double *) override { return fail_state("not available on a batch"); }
    int eta_bar(double *) override { return fail_state("not available on a batch"); }
    int attraction_potential(double *) override { return fail_state("not available on a batch"); }
    int get_pop(double *) override { return fail_state("not available on a batch"); }
    int set_pop(const double *) override { return fail_state("not available on a batch"); }

    int graph_steps_ = 10;

private:
    std::vector<hslb_params> p_;
    bool rows16_ = false;  // every slit 16 nodes wide in x (see launch_batch_collide)
    bool fused_rows_ = false;  // every slit's layer whole 256-node blocks of x-rows (phase 4)
    std::vector<SlitDesc> desc_;
    std::vector<WorkItem> wl_nodes_, wl_rows_, wl_fluid_, wl_prof_;
    std::vector<int> prof_off_;
    std::vector<char> inited_;
    int pop_stride_ = 0, fld_stride_ = 0, nprof_ = 0, ncu_ = 256, grid_per_cu_ = 8, cgrid_per_cu_ = 8, order_ = 0;
    int64_t nfluid_ = 0;
    hipStream_t stream_ = nullptr, ext_stream_ = nullptr;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    TF *f_[2] = {nullptr, nullptr};
    int cur_ = 0;
    TM *fld_mem_ = nullptr, *rs_ = nullptr;
    Fields<TM> fld_{};
    void *aux_ = nullptr;
    SlitDesc *desc_d_ = nullptr;
    WorkItem *work_d_ = nullptr;
    double *chi_d_ = nullptr, *prof_d_ = nullptr, *prof_h_ = nullptr, *io_d_ = nullptr;
    int *prof_off_d_ = nullptr;
    size_t io_bytes_ = 0;
    int64_t last_steps_ = 0;
    bool prof_valid_ = false, capturing_ = false;
    hipGraphExec_t gexec_[2] = {nullptr, nullptr};
    double *nref_d_ = nullptr;  // [2][sum nz][19]: read tables, write tables
    int ztot_ = 0;
    int64_t refreshed_at_ = -1;
};

const char *g_static_err = "invalid context";
thread_local std::string g_create_err;

}  // namespace

struct hslb_ctx {
    hslb_params p;
    std::unique_ptr<Engine> eng;
    std::string err;
};

static int validate(const hslb_params *p, std::string &err)
{
    if (!p) return fail(err, HSLB_EINVAL, "null parameters");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(err, HSLB_EINVAL, "grid sizes must be >= 1");
    if (p->wall_lo < 0 || p->wall_hi < 0 || ((p->wall_lo == 0) != (p->wall_hi == 0)))
        return fail(err, HSLB_EINVAL, "walls: both 0 (z periodic) or both >= 1");
    if (p->wall_lo + p->wall_hi >= p->nz) return fail(err, HSLB_EINVAL, "no fluid layer between the walls");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(err, HSLB_EINVAL, "tau must exceed 1/2");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->accel[a])) return fail(err, HSLB_EINVAL, "accel must be finite");
    if (p->precision != HSLB_FP32 && p->precision != HSLB_FP64) return fail(err, HSLB_EINVAL, "precision");
    if (p->g2_model != HSLB_G2_PAPER && p->g2_model != HSLB_G2_CS) return fail(err, HSLB_EINVAL, "g2_model");
    if (p->force_mode < 0 || p->force_mode > 2) return fail(err, HSLB_EINVAL, "force_mode");
    if (p->force_mode != HSLB_FORCE_OFF) {
        if (p->sigma < 2 || p->sigma > 8) return fail(err, HSLB_EINVAL, "sigma must be in 2..8");
        if (p->nx < p->sigma + 2 || p->ny < p->sigma + 2)
            return fail(err, HSLB_EINVAL, "nx and ny must be >= sigma + 2");
    } else if (p->nx < 2 || p->ny < 2) {
        return fail(err, HSLB_EINVAL, "nx and ny must be >= 2");
    }
    if (p->force_mode == HSLB_FORCE_SURROGATE) {
        if (p->nx % 32 || p->ny % 4)
            return fail(err, HSLB_EINVAL, "the learned force needs nx %% 32 == 0 and ny %% 4 == 0");
        if (p->surr_check_every < 1) return fail(err, HSLB_EINVAL, "surr_check_every must be >= 1");
        if (!(p->surr_tol > 0.0)) return fail(err, HSLB_EINVAL, "surr_tol must be > 0");
    }
    if (!std::isfinite(p->att_eps)) return fail(err, HSLB_EINVAL, "att_eps must be finite");
    if (p->att_eps != 0.0) {
        if (!(p->att_range > 0.0 && p->att_range <= 10.0))
            return fail(err, HSLB_EINVAL, "att_range must be in (0, 10] with the attraction on");
        if (p->force_mode == HSLB_FORCE_SURROGATE)
            return fail(err, HSLB_EINVAL, "the attraction is not available with the learned force");
    }
    if (p->lattice != HSLB_D3Q19 && p->lattice != HSLB_D3Q39) return fail(err, HSLB_EINVAL, "lattice");
    if (p->thermal != 0 && p->thermal != 1) return fail(err, HSLB_EINVAL, "thermal");
    if (p->thermal && p->lattice != HSLB_D3Q39)
        return fail(err, HSLB_EINVAL, "the non-isothermal terms need the 39-velocity lattice");
    if (p->lattice == HSLB_D3Q39) {
        if (p->precision != HSLB_FP64) return fail(err, HSLB_EINVAL, "the 39-velocity lattice is FP64 only");
        if (p->force_mode == HSLB_FORCE_SURROGATE)
            return fail(err, HSLB_EINVAL, "the learned force needs the 19-velocity lattice");
        if (p->nx < 3 || p->ny < 3) return fail(err, HSLB_EINVAL, "the 39-velocity lattice needs nx, ny >= 3");
        if (p->wall_lo == 0 && p->nz < 3) return fail(err, HSLB_EINVAL, "the 39-velocity lattice needs nz >= 3");
        if (p->wall_lo > 0 && p->nz - p->wall_lo - p->wall_hi < 3)
            return fail(err, HSLB_EINVAL, "the 39-velocity lattice needs at least 3 fluid layers");
    }
    const int sig = p->sigma >= 2 ? p->sigma : 2;
    const double fld = (double)p->nx * p->ny * (p->nz + 2.0 * sig);
    if (fld + 64 >= 2147483647.0) return fail(err, HSLB_EINVAL, "grid too large for 32-bit node indices");
    return HSLB_OK;
}

namespace hslb {
int context_training_pair(hslb_ctx *ctx, uint16_t *x, float *target, cnn::Geo *g, int *wall_lo, int *wall_hi,
                          int *sigma, std::string *msg);
}

extern "C" {

int hslb_create(const hslb_params *p, hslb_ctx **out)
{
    if (!out) return HSLB_EINVAL;
    std::string &err = g_create_err;
    err.clear();
    int rc = validate(p, err);
    if (rc) return rc;
    std::unique_ptr<hslb_ctx> c(new (std::nothrow) hslb_ctx());
    if (!c) return fail(err, HSLB_ENOMEM, "context allocation");
    c->p = *p;
    if (p->precision == HSLB_FP32) {
        auto e = std::make_unique<EngineT<float, float>>(*p);
        rc = e->setup();
        c->eng = std::move(e);
    } else {
        auto e = std::make_unique<EngineT<double, double>>(*p);
        rc = e->setup();
        c->eng = std::move(e);
    }
    if (rc) {
        err = c->eng->err;
        return rc;
    }
    // a diverging run stops with HSLB_EUNSTABLE instead of stepping on in NaNs
    c->eng->watch_every = kWatchEvery;
    c->eng->watch_tol = kWatchTol;
    *out = c.release();
    return HSLB_OK;
}

void hslb_destroy(hslb_ctx *ctx) { delete ctx; }

const char *hslb_last_error(const hslb_ctx *ctx)
{
    if (!ctx) return g_create_err.empty() ? g_static_err : g_create_err.c_str();
    if (!ctx->eng) return g_static_err;
    return ctx->eng->err.c_str();
}

#define CTX_CHECK(ctx)                                     \
    do {                                                   \
        if (!(ctx) || !(ctx)->eng) return HSLB_EINVAL;     \
    } while (0)

int hslb_set_stream(hslb_ctx *ctx, void *s)
{
    CTX_CHECK(ctx);
    ctx->eng->set_stream((hipStream_t)s);
    return HSLB_OK;
}

int hslb_init(hslb_ctx *ctx, const double *n, const double *u)
{
    CTX_CHECK(ctx);
    if (!n) return fail(ctx->eng->err, HSLB_EINVAL, "null density");
    return ctx->eng->init(n, u);
}

int hslb_init_thermal(hslb_ctx *ctx, const double *n, const double *u, const double *T)
{
    CTX_CHECK(ctx);
    if (!n) return fail(ctx->eng->err, HSLB_EINVAL, "null density");
    return ctx->eng->init_thermal(n, u, T);
}

int hslb_thermal_fields(hslb_ctx *ctx, double *T, double *Q)
{
    CTX_CHECK(ctx);
    if (!T && !Q) return fail(ctx->eng->err, HSLB_EINVAL, "null outputs");
    return ctx->eng->thermal_fields(T, Q);
}

int hslb_step(hslb_ctx *ctx, int64_t nsteps)
{
    CTX_CHECK(ctx);
    return ctx->eng->step(nsteps);
}

int hslb_sync(hslb_ctx *ctx)
{
    CTX_CHECK(ctx);
    return ctx->eng->sync();
}

int hslb_prepare(hslb_ctx *ctx)
{
    CTX_CHECK(ctx);
    return ctx->eng->prepare();
}

int hslb_step_count(const hslb_ctx *ctx, int64_t *s)
{
    if (!ctx || !ctx->eng || !s) return HSLB_EINVAL;
    *s = ctx->eng->steps;
    return HSLB_OK;
}

int hslb_moments(hslb_ctx *ctx, double *n, double *u)
{
    CTX_CHECK(ctx);
    return ctx->eng->moments(n, u);
}

int hslb_profiles(hslb_ctx *ctx, double *n_z, double *u_z)
{
    CTX_CHECK(ctx);
    return ctx->eng->profiles(n_z, u_z);
}

int hslb_force(hslb_ctx *ctx, double *F)
{
    CTX_CHECK(ctx);
    if (!F) return fail(ctx->eng->err, HSLB_EINVAL, "null output");
    return ctx->eng->force(F);
}

int hslb_eta_bar(hslb_ctx *ctx, double *eb)
{
    CTX_CHECK(ctx);
    if (!eb) return fail(ctx->eng->err, HSLB_EINVAL, "null output");
    if (ctx->p.force_mode == HSLB_FORCE_OFF) return fail(ctx->eng->err, HSLB_ESTATE, "hard-sphere term is off");
    return ctx->eng->eta_bar(eb);
}

int hslb_set_solid(hslb_ctx *ctx, const uint8_t *solid)
{
    CTX_CHECK(ctx);
    if (!solid) return fail(ctx->eng->err, HSLB_EINVAL, "null mask");
    return ctx->eng->set_solid(solid);
}

int hslb_attraction_potential(hslb_ctx *ctx, double *phi)
{
    CTX_CHECK(ctx);
    if (!phi) return fail(ctx->eng->err, HSLB_EINVAL, "null output");
    return ctx->eng->attraction_potential(phi);
}

int hslb_get_populations(hslb_ctx *ctx, double *f)
{
    CTX_CHECK(ctx);
    if (!f) return fail(ctx->eng->err, HSLB_EINVAL, "null output");
    return ctx->eng->get_pop(f);
}

int hslb_set_populations(hslb_ctx *ctx, const double *f)
{
    CTX_CHECK(ctx);
    if (!f) return fail(ctx->eng->err, HSLB_EINVAL, "null input");
    return ctx->eng->set_pop(f);
}

int hslb_set_watchdog(hslb_ctx *ctx, int64_t every, double tol)
{
    CTX_CHECK(ctx);
    if (every < 0 || !(tol >= 0.0)) return fail(ctx->eng->err, HSLB_EINVAL, "watchdog parameters");
    ctx->eng->watch_every = every;
    ctx->eng->watch_tol = tol;
    return HSLB_OK;
}

int hslb_checkpoint_size(hslb_ctx *ctx, int64_t *bytes)
{
    CTX_CHECK(ctx);
    if (!bytes) return fail(ctx->eng->err, HSLB_EINVAL, "null output");
    return ctx->eng->checkpoint_bytes(bytes);
}

int hslb_checkpoint_save(hslb_ctx *ctx, void *buf)
{
    CTX_CHECK(ctx);
    if (!buf) return fail(ctx->eng->err, HSLB_EINVAL, "null buffer");
    return ctx->eng->checkpoint_save(buf);
}

int hslb_checkpoint_load(hslb_ctx *ctx, const void *buf)
{
    CTX_CHECK(ctx);
    if (!buf) return fail(ctx->eng->err, HSLB_EINVAL, "null buffer");
    return ctx->eng->checkpoint_load(buf);
}

int hslb_surrogate_set_weights(hslb_ctx *ctx, const float *w, int64_t nw)
{
    CTX_CHECK(ctx);
    if (!w) return fail(ctx->eng->err, HSLB_EINVAL, "null weights");
    if (nw != cnn::NW) return fail(ctx->eng->err, HSLB_EINVAL, "expected %d weights, got %lld", cnn::NW, (long long)nw);
    return ctx->eng->surr_set_weights(w);
}

int hslb_surrogate_get_weights(hslb_ctx *ctx, float *w, int64_t nw)
{
    CTX_CHECK(ctx);
    if (!w) return fail(ctx->eng->err, HSLB_EINVAL, "null weights");
    if (nw != cnn::NW) return fail(ctx->eng->err, HSLB_EINVAL, "expected %d weights, got %lld", cnn::NW, (long long)nw);
    return ctx->eng->surr_get_weights(w);
}

int hslb_surrogate_set_mode(hslb_ctx *ctx, int32_t mode)
{
    CTX_CHECK(ctx);
    return ctx->eng->surr_set_mode(mode);
}

int hslb_surrogate_set_components(hslb_ctx *ctx, int32_t mask)
{
    CTX_CHECK(ctx);
    return ctx->eng->surr_set_components(mask);
}

int hslb_surrogate_stats(hslb_ctx *ctx, int64_t *checks, int64_t *fallback_steps, double *last_residual,
                         double *max_residual)
{
    CTX_CHECK(ctx);
    return ctx->eng->surr_stats(checks, fallback_steps, last_residual, max_residual);
}

int hslb_surrogate_force(hslb_ctx *ctx, double *F)
{
    CTX_CHECK(ctx);
    if (!F) return fail(ctx->eng->err, HSLB_EINVAL, "null output");
    return ctx->eng->surr_force(F);
}

int hslb_set_shift_period(hslb_ctx *ctx, int64_t every)
{
    CTX_CHECK(ctx);
    if (every < 0) return fail(ctx->eng->err, HSLB_EINVAL, "negative period");
    ctx->eng->shift_every = every;
    return HSLB_OK;
}

int hslb_set_graph(hslb_ctx *ctx, int32_t enable)
{
    CTX_CHECK(ctx);
    ctx->eng->use_graph = enable != 0;
    return HSLB_OK;
}

int hslb_set_collide_tiles(hslb_ctx *ctx, int32_t enable)
{
    CTX_CHECK(ctx);
    return ctx->eng->set_collide_tiles(enable != 0);
}

int hslb_set_kernel_timing(hslb_ctx *ctx, int32_t enable)
{
    CTX_CHECK(ctx);
    ctx->eng->kt.enabled = enable != 0;
    ctx->eng->kt.totals.clear();
    return HSLB_OK;
}

int hslb_kernel_times(hslb_ctx *ctx, int32_t cap, char (*names)[32], double *total_ms, int64_t *launches,
                      int32_t *count)
{
    CTX_CHECK(ctx);
    int32_t k = 0;
    for (auto &t : ctx->eng->kt.totals) {
        if (k < cap) {
            if (names) {
                std::strncpy(names[k], t.first.c_str(), 31);
                names[k][31] = 0;
            }
            if (total_ms) total_ms[k] = t.second.first;
            if (launches) launches[k] = t.second.second;
        }
        ++k;
    }
    if (count) *count = k;
    return HSLB_OK;
}

int hslb_get_timings(hslb_ctx *ctx, double *ms_per_step, double *mlups)
{
    CTX_CHECK(ctx);
    return ctx->eng->timings(ms_per_step, mlups);
}

int hslb_batch_create(const hslb_params *slits, int32_t nslits, hslb_ctx **out)
{
    std::string &err = g_create_err;
    err.clear();
    if (!out || !slits || nslits < 1) return fail(err, HSLB_EINVAL, "batch arguments");
    for (int k = 0; k < nslits; ++k) {
        int rc = validate(&slits[k], err);
        if (rc) {
            err = "slit " + std::to_string(k) + ": " + err;
            return rc;
        }
        if (slits[k].precision != slits[0].precision) return fail(err, HSLB_EINVAL, "mixed precisions in a batch");
        if (slits[k].force_mode == HSLB_FORCE_SURROGATE) return fail(err, HSLB_EINVAL, "surrogate in a batch");
        if (slits[k].lattice != HSLB_D3Q19) return fail(err, HSLB_EINVAL, "a batch holds 19-velocity slits");
        if (slits[k].att_eps != 0.0) return fail(err, HSLB_EINVAL, "attraction in a batch");
    }
    std::unique_ptr<hslb_ctx> c(new (std::nothrow) hslb_ctx());
    if (!c) return fail(err, HSLB_ENOMEM, "context allocation");
    c->p = slits[0];
    std::vector<hslb_params> v(slits, slits + nslits);
    int rc;
    if (slits[0].precision == HSLB_FP32) {
        auto e = std::make_unique<BatchT<float, float>>(v);
        rc = e->setup();
        c->eng = std::move(e);
    } else {
        auto e = std::make_unique<BatchT<double, double>>(v);
        rc = e->setup();
        c->eng = std::move(e);
    }
    if (rc) {
        err = c->eng->err;
        return rc;
    }
    *out = c.release();
    return HSLB_OK;
}

int hslb_batch_init(hslb_ctx *ctx, int32_t slit, const double *n, const double *u)
{
    CTX_CHECK(ctx);
    if (!n) return fail(ctx->eng->err, HSLB_EINVAL, "null density");
    return ctx->eng->batch_init(slit, n, u);
}

int hslb_batch_profiles(hslb_ctx *ctx, int32_t slit, double *n_z, double *u_z)
{
    CTX_CHECK(ctx);
    return ctx->eng->batch_profiles(slit, n_z, u_z);
}

int hslb_batch_finite(hslb_ctx *ctx, int32_t *flags)
{
    CTX_CHECK(ctx);
    if (!flags) return fail(ctx->eng->err, HSLB_EINVAL, "null output");
    return ctx->eng->batch_finite(flags);
}

int hslb_batch_set_config(hslb_ctx *ctx, int32_t grid_per_cu, int32_t order)
{
    CTX_CHECK(ctx);
    return ctx->eng->batch_set_config(grid_per_cu, order);
}

int hslb_batch_set_launch(hslb_ctx *ctx, int32_t phase_grid_per_cu, int32_t collide_grid_per_cu, int32_t order)
{
    CTX_CHECK(ctx);
    return ctx->eng->batch_set_launch(phase_grid_per_cu, collide_grid_per_cu, order);
}

int hslb_batch_get_launch(hslb_ctx *ctx, int32_t *phase_grid_per_cu, int32_t *collide_grid_per_cu, int32_t *order)
{
    CTX_CHECK(ctx);
    return ctx->eng->batch_get_launch(phase_grid_per_cu, collide_grid_per_cu, order);
}

int hslb_batch_autotune(hslb_ctx *ctx, int32_t steps, int32_t *choice, double *us_per_step, int32_t cap)
{
    CTX_CHECK(ctx);
    if (steps < 1) return fail(ctx->eng->err, HSLB_EINVAL, "autotune steps");
    return ctx->eng->batch_autotune(steps, choice, us_per_step, cap);
}

static_assert(kScratchBytes == (size_t)HSLB_FORCE_NOALLOC_BYTES, "scratch size of the header");

int hslb_force_noalloc(const hslb_params *p, const double *n, const double *u, double *F, void *hip_stream)
{
    std::string &err = g_create_err;
    err.clear();
    int rc = validate(p, err);
    if (rc) return rc;
    if (p->precision != HSLB_FP64 || p->lattice != HSLB_D3Q19 || p->force_mode == HSLB_FORCE_SURROGATE ||
        p->att_eps != 0.0)
        return fail(err, HSLB_EINVAL, "hslb_force_noalloc takes FP64 19-velocity lattices, exact or no force, "
                                      "no attraction");
    if (!n || !F) return fail(err, HSLB_EINVAL, "null device pointer");
    LatticeDev L{};
    StepConst sc{};
    std::vector<double> chi_h;
    slit_consts(*p, L, sc, chi_h);
    const int sig = p->sigma >= 2 ? p->sigma : 2;
    L.pop_stride = L.N;  // the equilibrium kernel writes [19][N]
    L.fld_stride = (L.plane * (p->nz + 2 * L.hz) + 63) / 64 * 64;
    // scratch layout (doubles, each part 256-byte aligned): populations
    // [19][N], reference table [nz][19] (zeros), chi[nz], then n, (n, j) [4],
    // eta_bar, the 7 contact-value slots and sigma/2 + 1 row-sum fields
    auto al = [](size_t d) { return (d + 31) / 32 * 32; };
    const size_t o_ref = al((size_t)NQ * L.N), o_chi = o_ref + al((size_t)NQ * p->nz);
    const size_t o_fld = o_chi + al((size_t)p->nz);
    const size_t nfld = (size_t)(1 + 4 + 1 + NGSLOT + sig / 2 + 1) * L.fld_stride;
    const size_t need = sizeof(double) * (o_fld + nfld);
    if (need > kScratchBytes)
        return fail(err, HSLB_EINVAL, "lattice needs %zu bytes of scratch, more than the %zu the allocation-free "
                                      "entry point holds", need, kScratchBytes);
    void *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return fail(err, HSLB_EDEVICE, "scratch address: %s", hipGetErrorString(e));
    double *d = (double *)base;
    hipStream_t s = (hipStream_t)hip_stream;
    Fields<double> fld{};
    fld.n = d + o_fld;
    fld.nj = fld.n + L.fld_stride;
    fld.eb = fld.n + 5 * (size_t)L.fld_stride;
    fld.G = fld.n + 6 * (size_t)L.fld_stride;
    double *rs = fld.n + (size_t)(6 + NGSLOT) * L.fld_stride;
    // the scratch keeps the previous call's contents: clear the reference
    // table and every field (their padding layers must read zero)
#define NA_TRY(...)                                                                                        \
    do {                                                                                                   \
        hipError_t e_ = (__VA_ARGS__);                                                                     \
        if (e_ != hipSuccess) return fail(err, HSLB_EDEVICE, "%s: %s", #__VA_ARGS__, hipGetErrorString(e_)); \
    } while (0)
    NA_TRY(launch_fill(s, d + o_ref, (size_t)NQ * p->nz, 0.0));
    NA_TRY(launch_fill(s, fld.n, nfld, 0.0));
    NA_TRY(launch_chi(s, L, sig, p->wall_reg, d + o_chi));
    if (u) {
        NA_TRY(launch_feq(s, L, n, u, d));
    } else {
        // rest: the equilibrium of (n, 0) from a zero velocity field held in F
        NA_TRY(launch_fill(s, F, 3 * (size_t)L.N, 0.0));
        NA_TRY(launch_feq(s, L, n, F, d));
    }
    NA_TRY(launch_moments<double, double>(s, L, d + o_ref, d, fld));
    if (sc.hs_on) {
        NA_TRY(launch_smooth2<double>(s, L, sig, sc.eta_pref, fld, rs));
        NA_TRY(launch_gfield<double>(s, L, sc.g2_model, fld));
    }
    sc.nref_r = sc.nref_w = d + o_ref;
    NA_TRY(launch_force<double, double>(s, L, sig, sc, d + o_chi, d, fld, F));
#undef NA_TRY
    return HSLB_OK;
}

int hslb_copy_bandwidth(int64_t bytes, int32_t iters, double *gbps)
{
    std::string &err = g_create_err;
    if (bytes < 16 * 256 || iters < 1 || !gbps) return fail(err, HSLB_EINVAL, "copy probe arguments");
    bytes = bytes / 16 * 16;
    void *a = nullptr, *b = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = HSLB_OK;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        rc = fail(err, HSLB_ENOMEM, "copy probe buffers");
    } else if (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
               hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(a, 0, bytes, s) != hipSuccess ||
               launch_copy(s, a, b, bytes) != hipSuccess || hipEventRecord(e0, s) != hipSuccess) {
        rc = fail(err, HSLB_EDEVICE, "copy probe setup");
    } else {
        for (int k = 0; k < iters && rc == HSLB_OK; ++k)
            if (launch_copy(s, a, b, bytes) != hipSuccess) rc = fail(err, HSLB_EDEVICE, "copy launch");
        float ms = 0.f;
        if (rc == HSLB_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = fail(err, HSLB_EDEVICE, "copy probe timing");
        if (rc == HSLB_OK) *gbps = 2.0 * (double)bytes * iters / (ms * 1e-3) / 1e9;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}

}  // extern "C"

namespace hslb {
int context_training_pair(hslb_ctx *ctx, uint16_t *x, float *target, cnn::Geo *g, int *wall_lo, int *wall_hi,
                          int *sigma, std::string *msg)
{
    if (!ctx || !ctx->eng) return HSLB_EINVAL;
    const int rc = ctx->eng->training_pair(x, target, g, wall_lo, wall_hi, sigma);
    if (rc && msg) *msg = ctx->eng->err;
    return rc;
}

// Records a failure of a call made on ctx from another translation unit.
int context_fail(hslb_ctx *ctx, int code, const std::string &msg)
{
    if (ctx && ctx->eng) ctx->eng->err = msg;
    return code;
}
}  // namespace hslb
