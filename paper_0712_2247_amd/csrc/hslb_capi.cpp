// Host engine and C ABI of libhslb.so (declared in include/hslb.h).
//
// The engine owns every device buffer of one lattice, builds the per-sigma
// constants in FP64 on the host, sequences the kernels of a time step on one
// HIP stream, replays pairs of steps from captured HIP graphs, and copies
// results out on request.
#include "hslb.h"
#include "hslb_internal.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

using namespace hslb;

namespace {

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
    virtual int get_pop(double *f) = 0;
    virtual int set_pop(const double *f) = 0;
    virtual int sync() = 0;
    virtual int timings(double *ms, double *mlups) = 0;
    virtual void set_stream(hipStream_t s) = 0;
    std::string err;
    int64_t steps = 0;
    bool inited = false;
    int64_t watch_every = 0;
    double watch_tol = 0.0;
    bool use_graph = true;
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
        for (int k = 0; k < 2; ++k)
            if (gexec_[k]) (void)hipGraphExecDestroy(gexec_[k]);
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
        (void)hipFree(f_[0]);
        (void)hipFree(f_[1]);
        (void)hipFree(fld_mem_);
        (void)hipFree(chi_d_);
        (void)hipFree(prof_d_);
        (void)hipHostFree(prof_h_);
        (void)hipFree(io_d_);
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

        sc_.tau = p_.tau;
        for (int a = 0; a < 3; ++a) sc_.g[a] = p_.accel[a];
        sc_.n_ref = 0.0;
        const double vt2 = 1.0 / 3.0;
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
        const size_t popb = sizeof(TF) * (size_t)NQ * L_.pop_stride;
        if (hipMalloc(&f_[0], popb) != hipSuccess || hipMalloc(&f_[1], popb) != hipSuccess)
            return fail(err, HSLB_ENOMEM, "population buffers (%zu bytes each) do not fit", popb);
        // n, j, eta_bar, the 7 contact-value slots and sigma/2 + 1 row-sum fields
        const size_t nfld = (size_t)(1 + 3 + 1 + NGSLOT + sig / 2 + 1) * L_.fld_stride;
        if (hipMalloc(&fld_mem_, sizeof(TM) * nfld) != hipSuccess)
            return fail(err, HSLB_ENOMEM, "moment fields do not fit");
        HIP_TRY(hipMemset(fld_mem_, 0, sizeof(TM) * nfld));
        HIP_TRY(hipMemset(f_[0], 0, popb));
        HIP_TRY(hipMemset(f_[1], 0, popb));
        fld_.n = fld_mem_;
        fld_.j = fld_mem_ + L_.fld_stride;
        fld_.eb = fld_mem_ + 4 * (size_t)L_.fld_stride;
        fld_.G = fld_mem_ + 5 * (size_t)L_.fld_stride;
        rs_ = fld_mem_ + (size_t)(5 + NGSLOT) * L_.fld_stride;

        std::vector<double> chi(p_.nz, 1.0);
        if (!L_.zper && p_.wall_reg) {
            const double za = p_.wall_lo - 0.5, zb = p_.nz - p_.wall_hi - 0.5;
            for (int z = 0; z < p_.nz; ++z) {
                const double dw = std::fmin((double)z - za, zb - (double)z);
                chi[z] = 1.0 - std::exp(-dw / (double)sig);
            }
        }
        HIP_TRY(hipMalloc(&chi_d_, sizeof(double) * p_.nz));
        HIP_TRY(hipMemcpy(chi_d_, chi.data(), sizeof(double) * p_.nz, hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc(&prof_d_, sizeof(double) * 5 * p_.nz));
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

    void drop_graphs()
    {
        for (int k = 0; k < 2; ++k)
            if (gexec_[k]) {
                (void)hipGraphExecDestroy(gexec_[k]);
                gexec_[k] = nullptr;
            }
    }

    int init(const double *n, const double *u) override
    {
        const int N = L_.N;
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
            msum += n[id];
            ++nfl;
        }
        sc_.n_ref = nfl ? msum / (double)nfl : 0.0;
        mass0_ = msum;
        double *d;
        int rc = io(sizeof(double) * 4 * (size_t)N, &d);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(d, n, sizeof(double) * N, hipMemcpyHostToDevice, st()));
        if (u)
            HIP_TRY(hipMemcpyAsync(d + N, u, sizeof(double) * 3 * (size_t)N, hipMemcpyHostToDevice, st()));
        else
            HIP_TRY(hipMemsetAsync(d + N, 0, sizeof(double) * 3 * (size_t)N, st()));
        cur_ = 0;
        HIP_TRY(launch_init<TF>(st(), L_, sc_.n_ref, d, d + N, f_[0]));
        HIP_TRY(hipStreamSynchronize(st()));
        drop_graphs();
        steps = 0;
        inited = true;
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

    int one_step()
    {
        int rc = launch("moments", [&] { return launch_moments<TF, TM>(st(), L_, sc_.n_ref, f_[cur_], fld_); });
        if (rc) return rc;
        if (sc_.hs_on && (rc = fields_hs())) return rc;
        rc = launch("collide", [&] {
            return launch_collide<TF, TM>(st(), L_, sigma_, sc_, chi_d_, f_[cur_], f_[1 - cur_], fld_);
        });
        if (rc) return rc;
        cur_ = 1 - cur_;
        return HSLB_OK;
    }

    int capture(int parity)
    {
        const int save = cur_;
        cur_ = parity;
        hipGraph_t g = nullptr;
        capturing_ = true;
        HIP_TRY(hipStreamBeginCapture(st(), hipStreamCaptureModeThreadLocal));
        int rc = one_step();
        if (!rc) rc = one_step();
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
        e = hipGraphInstantiate(&gexec_[parity], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(err, HSLB_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
        return HSLB_OK;
    }

    int advance(int64_t n)
    {
        const bool graph = use_graph && !kt.enabled;
        while (n > 0) {
            if (graph && n >= 2) {
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

    int watchdog_check()
    {
        HIP_TRY(launch_profiles_pop<TF>(st(), L_, sc_.n_ref, f_[cur_], prof_d_));
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
        HIP_TRY(launch_export_moments<TF>(st(), L_, sc_.n_ref, f_[cur_], d, d + N));
        if (n) HIP_TRY(hipMemcpyAsync(n, d, sizeof(double) * N, hipMemcpyDeviceToHost, st()));
        if (u) HIP_TRY(hipMemcpyAsync(u, d + N, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int profiles(double *nz, double *uz) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "profiles before init");
        HIP_TRY(launch_profiles_pop<TF>(st(), L_, sc_.n_ref, f_[cur_], prof_d_));
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
        HIP_TRY(launch_moments<TF, TM>(st(), L_, sc_.n_ref, f_[cur_], fld_));
        if (sc_.hs_on && (rc = fields_hs())) return rc;
        HIP_TRY(launch_force<TF, TM>(st(), L_, sigma_, sc_, chi_d_, f_[cur_], fld_, d));
        HIP_TRY(hipMemcpyAsync(F, d, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int eta_bar(double *eb) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "eta_bar before init");
        double *d;
        int rc = io(sizeof(double) * (size_t)L_.N, &d);
        if (rc) return rc;
        HIP_TRY(launch_moments<TF, TM>(st(), L_, sc_.n_ref, f_[cur_], fld_));
        HIP_TRY(launch_smooth2<TM>(st(), L_, sigma_, sc_.eta_pref, fld_, rs_));
        HIP_TRY(launch_unpad<TM>(st(), L_, fld_.eb, d));
        HIP_TRY(hipMemcpyAsync(eb, d, sizeof(double) * L_.N, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int get_pop(double *f) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "get_populations before init");
        double *d;
        const size_t tot = (size_t)NQ * L_.N;
        int rc = io(sizeof(double) * tot, &d);
        if (rc) return rc;
        HIP_TRY(launch_get_pop<TF>(st(), L_, sc_.n_ref, f_[cur_], d));
        HIP_TRY(hipMemcpyAsync(f, d, sizeof(double) * tot, hipMemcpyDeviceToHost, st()));
        HIP_TRY(hipStreamSynchronize(st()));
        return HSLB_OK;
    }

    int set_pop(const double *f) override
    {
        if (!inited) return fail(err, HSLB_ESTATE, "set_populations before init");
        const size_t tot = (size_t)NQ * L_.N;
        for (size_t k = 0; k < tot; ++k)
            if (!std::isfinite(f[k]))
                return fail(err, HSLB_EINVAL, "population %zu is not finite", k);
        double *d;
        int rc = io(sizeof(double) * tot, &d);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(d, f, sizeof(double) * tot, hipMemcpyHostToDevice, st()));
        HIP_TRY(launch_set_pop<TF>(st(), L_, sc_.n_ref, d, f_[cur_]));
        HIP_TRY(hipStreamSynchronize(st()));
        steps = 0;
        return HSLB_OK;
    }

private:
    hslb_params p_;
    LatticeDev L_{};
    StepConst sc_{};
    int sigma_ = 2;
    hipStream_t stream_ = nullptr, ext_stream_ = nullptr;
    bool own_stream_ = false;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    TF *f_[2] = {nullptr, nullptr};
    int cur_ = 0;
    TM *fld_mem_ = nullptr;
    TM *rs_ = nullptr;
    Fields<TM> fld_{};
    double *chi_d_ = nullptr, *prof_d_ = nullptr, *prof_h_ = nullptr;
    double *io_d_ = nullptr;
    size_t io_bytes_ = 0;
    double mass0_ = 0.0;
    int64_t last_steps_ = 0;
    hipGraphExec_t gexec_[2] = {nullptr, nullptr};
    bool capturing_ = false;
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
    if (p->force_mode == HSLB_FORCE_SURROGATE) return fail(err, HSLB_ENOSURR, "no surrogate weights loaded");
    const int sig = p->sigma >= 2 ? p->sigma : 2;
    const double fld = (double)p->nx * p->ny * (p->nz + 2.0 * sig);
    if (fld + 64 >= 2147483647.0) return fail(err, HSLB_EINVAL, "grid too large for 32-bit node indices");
    return HSLB_OK;
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

int hslb_set_graph(hslb_ctx *ctx, int32_t enable)
{
    CTX_CHECK(ctx);
    ctx->eng->use_graph = enable != 0;
    return HSLB_OK;
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
