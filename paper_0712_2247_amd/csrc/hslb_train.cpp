// Training of the learned force on the GPU, and single network operations on
// host data (C ABI of include/hslb.h).
//
// A trainer keeps a store of snapshots in device memory -- the network input
// x = bf16(pi sigma^3 n / 6) and the target C1 / force scale of a lattice
// state -- plus FP32 master weights, the Adam moments and the work buffers of
// one forward and backward pass.  A training step on one snapshot:
//   forward   z1 = conv(x) + b1, a1 = GELU(z1), z2, a2, F_hat
//   loss      mean over fluid nodes and components of (F_hat - target)^2
//   backward  dz2 = conv^T(dF) * GELU'(z2), dz1 = conv^T(dz2) * GELU'(z1),
//             weight gradients from the channel-major activation copies,
//             bias gradients as column sums
//   Adam      on the master weights, then the bf16 operand packs are rebuilt.
#include "hslb.h"
#include "hslb_cnn.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <dirent.h>
#include <new>
#include <string>
#include <vector>

using namespace hslb;
using namespace hslb::cnn;

namespace hslb {
// hslb_capi.cpp: network input and target of a context's current state.
int context_training_pair(hslb_ctx *ctx, uint16_t *x, float *target, Geo *g, int *wall_lo, int *wall_hi, int *sigma,
                          std::string *msg);
int context_fail(hslb_ctx *ctx, int code, const std::string &msg);
}

namespace {

int tfail(std::string &err, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return code;
}

#define T_TRY(...)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (__VA_ARGS__);                                                               \
        if (e_ != hipSuccess)                                                                        \
            return tfail(err, HSLB_EDEVICE, "%s failed: %s", #__VA_ARGS__, hipGetErrorString(e_));   \
    } while (0)

// Device buffers of one forward + backward pass over up to `nmax` nodes.
struct Work {
    size_t nmax = 0;
    void *mem = nullptr;
    uint16_t *a1 = nullptr, *a2 = nullptr, *a1T = nullptr, *a2T = nullptr;
    float *z1 = nullptr, *z2 = nullptr, *out = nullptr;
    uint16_t *d3cl = nullptr, *d3cm = nullptr, *dz2cl = nullptr, *dz2cm = nullptr, *dz1cm = nullptr;
    float *wpart = nullptr, *cpart = nullptr;
    double *lpart = nullptr, *lpart_h = nullptr;
    size_t nlpart = 0;

    ~Work()
    {
        (void)hipFree(mem);
        (void)hipHostFree(lpart_h);
    }

    int alloc(size_t n, std::string &err)
    {
        nmax = n;
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off += (bytes + 255) / 256 * 256;
            return o;
        };
        const size_t o_a1 = take(2 * 32 * n), o_a2 = take(2 * 32 * n), o_a1T = take(2 * 32 * n), o_a2T = take(2 * 32 * n);
        const size_t o_z1 = take(4 * 32 * n), o_z2 = take(4 * 32 * n), o_out = take(4 * 3 * n);
        const size_t o_d3cl = take(2 * 4 * n), o_d3cm = take(2 * 3 * n), o_dz2cl = take(2 * 32 * n),
                     o_dz2cm = take(2 * 32 * n), o_dz1cm = take(2 * 32 * n);
        // scratch sized for the largest lattice of nmax nodes with nx = 32
        const Geo g{32, 4, (int)((n + 127) / 128), 0, (int)n};
        size_t wp = 0;
        for (int l = 1; l <= 3; ++l) wp = std::max(wp, wgrad_partial_floats(g, l));
        const size_t o_wp = take(4 * wp);
        const size_t o_cp = take(4 * colsum_partial_floats(g, 32));
        nlpart = loss_blocks(g) + 64;
        const size_t o_lp = take(8 * nlpart);
        if (hipMalloc(&mem, off) != hipSuccess) return tfail(err, HSLB_ENOMEM, "training work buffers (%zu bytes)", off);
        char *b = (char *)mem;
        a1 = (uint16_t *)(b + o_a1);
        a2 = (uint16_t *)(b + o_a2);
        a1T = (uint16_t *)(b + o_a1T);
        a2T = (uint16_t *)(b + o_a2T);
        z1 = (float *)(b + o_z1);
        z2 = (float *)(b + o_z2);
        out = (float *)(b + o_out);
        d3cl = (uint16_t *)(b + o_d3cl);
        d3cm = (uint16_t *)(b + o_d3cm);
        dz2cl = (uint16_t *)(b + o_dz2cl);
        dz2cm = (uint16_t *)(b + o_dz2cm);
        dz1cm = (uint16_t *)(b + o_dz1cm);
        wpart = (float *)(b + o_wp);
        cpart = (float *)(b + o_cp);
        lpart = (double *)(b + o_lp);
        if (hipHostMalloc((void **)&lpart_h, 8 * nlpart, hipHostMallocDefault) != hipSuccess)
            return tfail(err, HSLB_ENOMEM, "pinned loss buffer");
        return HSLB_OK;
    }
};

// Packed bf16 operands of all five convolutions.
struct Packs {
    uint16_t *p[PK_COUNT] = {};
    void *mem = nullptr;
    ~Packs() { (void)hipFree(mem); }
    int alloc(std::string &err)
    {
        size_t tot = 0;
        for (int k = 0; k < PK_COUNT; ++k) tot += pack_elems(k);
        if (hipMalloc(&mem, 2 * tot) != hipSuccess) return tfail(err, HSLB_ENOMEM, "weight packs");
        uint16_t *q = (uint16_t *)mem;
        for (int k = 0; k < PK_COUNT; ++k) {
            p[k] = q;
            q += pack_elems(k);
        }
        return HSLB_OK;
    }
    hipError_t build(hipStream_t s, const float *w)
    {
        for (int k = 0; k < PK_COUNT; ++k) {
            hipError_t e = launch_pack(s, k, w, p[k]);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

// Forward through the three layers.  a1T/a2T (channel-major copies) and the
// pre-activations are written when `train`.
hipError_t forward(hipStream_t s, const Geo &g, const uint16_t *x, const float *w, const Packs &pk, Work &wk, bool train)
{
    FwdArgs a{};
    a.g = g;
    a.in = x;
    a.wp = pk.p[PK_F1];
    a.bias = w + OB1;
    a.out_cl = wk.a1;
    a.out_cm = train ? wk.a1T : nullptr;
    a.out_f32 = train ? wk.z1 : nullptr;
    hipError_t e = launch_conv_fwd(s, 1, 32, EPI_GELU, a);
    if (e != hipSuccess) return e;
    a.in = wk.a1;
    a.wp = pk.p[PK_F2];
    a.bias = w + OB2;
    a.out_cl = wk.a2;
    a.out_cm = train ? wk.a2T : nullptr;
    a.out_f32 = train ? wk.z2 : nullptr;
    if ((e = launch_conv_fwd(s, 32, 32, EPI_GELU, a)) != hipSuccess) return e;
    a.in = wk.a2;
    a.wp = pk.p[PK_F3];
    a.bias = w + OB3;
    a.out_cl = nullptr;
    a.out_cm = nullptr;
    a.out_f32 = wk.out;
    return launch_conv_fwd(s, 32, 3, EPI_OUT, a);
}

// Backward from the bf16 output gradient (wk.d3cl / d3cm) into grad[NW].
hipError_t backward(hipStream_t s, const Geo &g, const uint16_t *x, const Packs &pk, Work &wk, float *grad)
{
    FwdArgs a{};
    a.g = g;
    a.in = wk.d3cl;
    a.wp = pk.p[PK_D3];
    a.zsave = wk.z2;
    a.out_cl = wk.dz2cl;
    a.out_cm = wk.dz2cm;
    hipError_t e = launch_conv_fwd(s, 4, 32, EPI_DGELU, a);
    if (e != hipSuccess) return e;
    a.in = wk.dz2cl;
    a.wp = pk.p[PK_D2];
    a.zsave = wk.z1;
    a.out_cl = nullptr;
    a.out_cm = wk.dz1cm;
    if ((e = launch_conv_fwd(s, 32, 32, EPI_DGELU, a)) != hipSuccess) return e;
    if ((e = launch_wgrad(s, 3, g, wk.a2T, wk.d3cm, wk.wpart, grad + OW3)) != hipSuccess) return e;
    if ((e = launch_colsum(s, g, CO, wk.d3cm, wk.cpart, grad + OB3)) != hipSuccess) return e;
    if ((e = launch_wgrad(s, 2, g, wk.a1T, wk.dz2cm, wk.wpart, grad + OW2)) != hipSuccess) return e;
    if ((e = launch_colsum(s, g, CH, wk.dz2cm, wk.cpart, grad + OB2)) != hipSuccess) return e;
    if ((e = launch_wgrad(s, 1, g, x, wk.dz1cm, wk.wpart, grad + OW1)) != hipSuccess) return e;
    return launch_colsum(s, g, CH, wk.dz1cm, wk.cpart, grad + OB1);
}

bool geo_ok(int nx, int ny, int nz) { return nx >= 32 && nx % 32 == 0 && ny >= 4 && ny % 4 == 0 && nz >= 1; }

}  // namespace

struct Snapshot {
    Geo g;
    int wall_lo, wall_hi;
    size_t x_off, t_off;  // in the arena: x (bf16) and target (FP32 [3][N])
};

struct hslb_trainer {
    std::string err;
    hipStream_t stream = nullptr;
    size_t cap_nodes = 0, used_bytes = 0, cap_bytes = 0;
    char *arena = nullptr;
    std::vector<Snapshot> snaps;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    double *stage = nullptr;
    size_t stage_bytes = 0;
    Packs pk;
    Work wk;
    int t = 0;
    bool have_w = false;

    ~hslb_trainer()
    {
        (void)hipFree(arena);
        (void)hipFree(w);
        (void)hipFree(stage);
        if (stream) (void)hipStreamDestroy(stream);
    }

    int stage_buf(size_t bytes, double **out)
    {
        if (bytes > stage_bytes) {
            (void)hipFree(stage);
            stage = nullptr;
            stage_bytes = 0;
            if (hipMalloc(&stage, bytes) != hipSuccess) return tfail(err, HSLB_ENOMEM, "staging buffer");
            stage_bytes = bytes;
        }
        *out = stage;
        return HSLB_OK;
    }

    int reserve(size_t N, Snapshot &sn)
    {
        if (N > wk.nmax) return tfail(err, HSLB_EINVAL, "snapshot of %zu nodes exceeds the per-snapshot maximum %zu", N, wk.nmax);
        const size_t xb = (2 * N + 255) / 256 * 256, tb = (12 * N + 255) / 256 * 256;
        if (used_bytes + xb + tb > cap_bytes) return tfail(err, HSLB_ENOMEM, "snapshot store is full");
        sn.x_off = used_bytes;
        sn.t_off = used_bytes + xb;
        used_bytes += xb + tb;
        return HSLB_OK;
    }

    // forward (+ loss); returns the loss of snapshot k
    int run(int k, bool train, double *loss)
    {
        const Snapshot &sn = snaps[k];
        const uint16_t *x = (const uint16_t *)(arena + sn.x_off);
        const float *tg = (const float *)(arena + sn.t_off);
        T_TRY(forward(stream, sn.g, x, w, pk, wk, train));
        T_TRY(launch_loss(stream, sn.g, sn.wall_lo, sn.wall_hi, wk.out, tg, wk.d3cl, wk.d3cm, wk.lpart));
        if (train) T_TRY(backward(stream, sn.g, x, pk, wk, grad));
        const unsigned nb = loss_blocks(sn.g);
        T_TRY(hipMemcpyAsync(wk.lpart_h, wk.lpart, 8 * nb, hipMemcpyDeviceToHost, stream));
        T_TRY(hipStreamSynchronize(stream));
        double s = 0.0;
        for (unsigned i = 0; i < nb; ++i) s += wk.lpart_h[i];
        const double nf = (double)sn.g.nx * sn.g.ny * (sn.g.nz - sn.wall_lo - sn.wall_hi);
        if (loss) *loss = s / (3.0 * nf);
        return HSLB_OK;
    }
};

namespace {
std::string g_trainer_err;
}

extern "C" {

int hslb_trainer_create(int64_t capacity_nodes, int64_t max_snapshot_nodes, hslb_trainer **out)
{
    if (!out) return HSLB_EINVAL;
    std::string &err = g_trainer_err;
    if (capacity_nodes < 1 || max_snapshot_nodes < 1 || max_snapshot_nodes > capacity_nodes)
        return tfail(err, HSLB_EINVAL, "capacity must be >= the per-snapshot maximum >= 1");
    if (max_snapshot_nodes >= (int64_t)1 << 26) return tfail(err, HSLB_EINVAL, "snapshots above 2^26 nodes");
    hslb_trainer *tr = new (std::nothrow) hslb_trainer();
    if (!tr) return tfail(err, HSLB_ENOMEM, "trainer allocation");
    int rc = HSLB_OK;
    auto bail = [&](int code) {
        err = tr->err;
        delete tr;
        return code;
    };
    if (hipStreamCreate(&tr->stream) != hipSuccess) return bail(tfail(tr->err, HSLB_EDEVICE, "stream"));
    tr->cap_nodes = (size_t)capacity_nodes;
    tr->cap_bytes = (size_t)capacity_nodes * 14 + 512 * 64;
    if (hipMalloc(&tr->arena, tr->cap_bytes) != hipSuccess)
        return bail(tfail(tr->err, HSLB_ENOMEM, "snapshot store of %zu bytes", tr->cap_bytes));
    if (hipMalloc(&tr->w, sizeof(float) * 4 * NW) != hipSuccess) return bail(tfail(tr->err, HSLB_ENOMEM, "weights"));
    tr->m = tr->w + NW;
    tr->v = tr->m + NW;
    tr->grad = tr->v + NW;
    if ((rc = tr->pk.alloc(tr->err))) return bail(rc);
    if ((rc = tr->wk.alloc((size_t)max_snapshot_nodes, tr->err))) return bail(rc);
    *out = tr;
    return HSLB_OK;
}

void hslb_trainer_destroy(hslb_trainer *tr) { delete tr; }

const char *hslb_trainer_last_error(const hslb_trainer *tr) { return tr ? tr->err.c_str() : g_trainer_err.c_str(); }

int hslb_trainer_add_snapshot(hslb_trainer *tr, hslb_ctx *ctx, int32_t *index)
{
    if (!tr || !ctx) return HSLB_EINVAL;
    std::string &err = tr->err;
    Geo g{};
    int wl = 0, wh = 0, sig = 0;
    int rc = context_training_pair(ctx, nullptr, nullptr, &g, &wl, &wh, &sig, &err);  // geometry only
    if (rc) return rc;
    if (!geo_ok(g.nx, g.ny, g.nz)) return tfail(err, HSLB_EINVAL, "snapshots need nx %% 32 == 0 and ny %% 4 == 0");
    Snapshot sn{};
    const size_t save = tr->used_bytes;
    if ((rc = tr->reserve((size_t)g.N, sn))) return rc;
    rc = context_training_pair(ctx, (uint16_t *)(tr->arena + sn.x_off), (float *)(tr->arena + sn.t_off), &g, &wl, &wh,
                               &sig, &err);
    if (rc) {
        tr->used_bytes = save;
        return rc;
    }
    sn.g = g;
    sn.wall_lo = wl;
    sn.wall_hi = wh;
    tr->snaps.push_back(sn);
    if (index) *index = (int32_t)tr->snaps.size() - 1;
    return HSLB_OK;
}

int hslb_trainer_add_snapshot_host(hslb_trainer *tr, int32_t nx, int32_t ny, int32_t nz, int32_t wall_lo,
                                   int32_t wall_hi, const double *eta, const double *target, int32_t *index)
{
    if (!tr || !eta || !target) return HSLB_EINVAL;
    std::string &err = tr->err;
    if (!geo_ok(nx, ny, nz)) return tfail(err, HSLB_EINVAL, "snapshots need nx %% 32 == 0 and ny %% 4 == 0");
    if (wall_lo < 0 || wall_hi < 0 || wall_lo + wall_hi >= nz || ((wall_lo == 0) != (wall_hi == 0)))
        return tfail(err, HSLB_EINVAL, "walls");
    Snapshot sn{};
    sn.g = Geo{nx, ny, nz, wall_lo == 0 ? 1 : 0, nx * ny * nz};
    sn.wall_lo = wall_lo;
    sn.wall_hi = wall_hi;
    const size_t N = (size_t)sn.g.N;
    int rc = tr->reserve(N, sn);
    if (rc) return rc;
    double *d;
    if ((rc = tr->stage_buf(8 * 4 * N, &d))) return rc;
    T_TRY(hipMemcpyAsync(d, eta, 8 * N, hipMemcpyHostToDevice, tr->stream));
    T_TRY(hipMemcpyAsync(d + N, target, 8 * 3 * N, hipMemcpyHostToDevice, tr->stream));
    T_TRY(launch_to_bf16(tr->stream, d, N, (uint16_t *)(tr->arena + sn.x_off)));
    T_TRY(launch_scale_f64_to_f32(tr->stream, d + N, 1.0, 3 * N, (float *)(tr->arena + sn.t_off)));
    T_TRY(hipStreamSynchronize(tr->stream));
    tr->snaps.push_back(sn);
    if (index) *index = (int32_t)tr->snaps.size() - 1;
    return HSLB_OK;
}

int hslb_trainer_count(hslb_trainer *tr, int32_t *count)
{
    if (!tr || !count) return HSLB_EINVAL;
    *count = (int32_t)tr->snaps.size();
    return HSLB_OK;
}

int hslb_trainer_set_weights(hslb_trainer *tr, const float *w, int64_t nw)
{
    if (!tr || !w) return HSLB_EINVAL;
    std::string &err = tr->err;
    if (nw != NW) return tfail(err, HSLB_EINVAL, "expected %d weights, got %lld", NW, (long long)nw);
    for (int i = 0; i < NW; ++i)
        if (!std::isfinite(w[i])) return tfail(err, HSLB_EINVAL, "weight %d is not finite", i);
    T_TRY(hipMemcpyAsync(tr->w, w, sizeof(float) * NW, hipMemcpyHostToDevice, tr->stream));
    T_TRY(hipMemsetAsync(tr->m, 0, sizeof(float) * 2 * NW, tr->stream));
    T_TRY(tr->pk.build(tr->stream, tr->w));
    T_TRY(hipStreamSynchronize(tr->stream));
    tr->t = 0;
    tr->have_w = true;
    return HSLB_OK;
}

int hslb_trainer_get_weights(hslb_trainer *tr, float *w, int64_t nw)
{
    if (!tr || !w) return HSLB_EINVAL;
    std::string &err = tr->err;
    if (nw != NW) return tfail(err, HSLB_EINVAL, "expected %d weights", NW);
    if (!tr->have_w) return tfail(err, HSLB_ENOSURR, "no weights set");
    T_TRY(hipMemcpyAsync(w, tr->w, sizeof(float) * NW, hipMemcpyDeviceToHost, tr->stream));
    T_TRY(hipStreamSynchronize(tr->stream));
    return HSLB_OK;
}

#define TR_CHECK(tr, k)                                                                                    \
    if (!tr) return HSLB_EINVAL;                                                                           \
    if (!tr->have_w) return tfail(tr->err, HSLB_ENOSURR, "no weights set");                                \
    if (k < 0 || k >= (int32_t)tr->snaps.size()) return tfail(tr->err, HSLB_EINVAL, "no snapshot %d", (int)k)

int hslb_trainer_eval(hslb_trainer *tr, int32_t k, double *loss, float *out)
{
    TR_CHECK(tr, k);
    std::string &err = tr->err;
    int rc = tr->run(k, false, loss);
    if (rc) return rc;
    if (out) {
        T_TRY(hipMemcpyAsync(out, tr->wk.out, sizeof(float) * 3 * (size_t)tr->snaps[k].g.N, hipMemcpyDeviceToHost,
                             tr->stream));
        T_TRY(hipStreamSynchronize(tr->stream));
    }
    return HSLB_OK;
}

int hslb_trainer_grad(hslb_trainer *tr, int32_t k, double *loss, float *grad)
{
    TR_CHECK(tr, k);
    std::string &err = tr->err;
    int rc = tr->run(k, true, loss);
    if (rc) return rc;
    if (grad) {
        T_TRY(hipMemcpyAsync(grad, tr->grad, sizeof(float) * NW, hipMemcpyDeviceToHost, tr->stream));
        T_TRY(hipStreamSynchronize(tr->stream));
    }
    return HSLB_OK;
}

int hslb_trainer_step(hslb_trainer *tr, int32_t k, double lr, double *loss)
{
    TR_CHECK(tr, k);
    std::string &err = tr->err;
    if (!(lr > 0.0) || !std::isfinite(lr)) return tfail(err, HSLB_EINVAL, "learning rate must be > 0");
    int rc = tr->run(k, true, loss);
    if (rc) return rc;
    tr->t += 1;
    T_TRY(launch_adam(tr->stream, NW, tr->w, tr->m, tr->v, tr->grad, tr->t, (float)lr));
    T_TRY(tr->pk.build(tr->stream, tr->w));
    return HSLB_OK;
}

int hslb_trainer_train(hslb_trainer *tr, const int32_t *order, int32_t n, double lr, double *mean_loss)
{
    if (!tr || (!order && n > 0) || n < 0) return HSLB_EINVAL;
    std::string &err = tr->err;
    if (!tr->have_w) return tfail(err, HSLB_ENOSURR, "no weights set");
    if (!(lr > 0.0) || !std::isfinite(lr)) return tfail(err, HSLB_EINVAL, "learning rate must be > 0");
    for (int32_t i = 0; i < n; ++i)
        if (order[i] < 0 || order[i] >= (int32_t)tr->snaps.size())
            return tfail(err, HSLB_EINVAL, "order[%d] = %d is not a snapshot", (int)i, (int)order[i]);
    double sum = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double L = 0.0;
        int rc = tr->run(order[i], true, &L);
        if (rc) return rc;
        if (!std::isfinite(L)) return tfail(err, HSLB_EUNSTABLE, "loss is not finite at step %d", (int)i);
        sum += L;
        tr->t += 1;
        T_TRY(launch_adam(tr->stream, NW, tr->w, tr->m, tr->v, tr->grad, tr->t, (float)lr));
        T_TRY(tr->pk.build(tr->stream, tr->w));
    }
    T_TRY(hipStreamSynchronize(tr->stream));
    if (mean_loss) *mean_loss = n > 0 ? sum / n : 0.0;
    return HSLB_OK;
}

int hslb_cnn_op(int32_t op, int32_t nx, int32_t ny, int32_t nz, int32_t zper, const float *w, const float *in,
                const float *aux, float *out)
{
    std::string &err = g_trainer_err;
    if (!w || !in || !out) return tfail(err, HSLB_EINVAL, "null argument");
    if (op < HSLB_CNN_FWD1 || op > HSLB_CNN_DW3) return tfail(err, HSLB_EINVAL, "operation %d", (int)op);
    if (!geo_ok(nx, ny, nz)) return tfail(err, HSLB_EINVAL, "needs nx %% 32 == 0 and ny %% 4 == 0");
    const bool need_aux = op >= HSLB_CNN_DX3;
    if (need_aux && !aux) return tfail(err, HSLB_EINVAL, "operation %d needs aux", (int)op);
    const Geo g{nx, ny, nz, zper ? 1 : 0, nx * ny * nz};
    const size_t N = (size_t)g.N;
    hipStream_t s = nullptr;
    T_TRY(hipStreamCreate(&s));
    struct Guard {
        hipStream_t s;
        std::vector<void *> bufs;
        ~Guard()
        {
            for (void *b : bufs) (void)hipFree(b);
            if (s) (void)hipStreamDestroy(s);
        }
        void *get(size_t bytes)
        {
            void *p = nullptr;
            if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
            bufs.push_back(p);
            return p;
        }
    } gd{s, {}};
    float *wd = (float *)gd.get(sizeof(float) * NW);
    Packs pk;
    int rc = pk.alloc(err);
    if (rc) return rc;
    const int cin = op == HSLB_CNN_FWD1 || op == HSLB_CNN_DW1 ? 1 : (op == HSLB_CNN_DX3 || op == HSLB_CNN_DW3 ? 3 : 32);
    // DW3 reads a2 (32 channels) with aux g3 (3); DX3 reads g3 (3) with aux z2 (32)
    const int c_in = op == HSLB_CNN_DW3 ? 32 : cin;
    const int c_aux = op == HSLB_CNN_DW3 ? 3 : (op == HSLB_CNN_DW1 ? 32 : 32);
    float *ind = (float *)gd.get(sizeof(float) * c_in * N);
    float *auxd = need_aux ? (float *)gd.get(sizeof(float) * c_aux * N) : nullptr;
    uint16_t *in_cl = (uint16_t *)gd.get(2 * 32 * N), *in_cm = (uint16_t *)gd.get(2 * 32 * N);
    uint16_t *aux_cm = (uint16_t *)gd.get(2 * 32 * N);
    float *f1 = (float *)gd.get(4 * 32 * N);
    uint16_t *b1 = (uint16_t *)gd.get(2 * 32 * N), *b2 = (uint16_t *)gd.get(2 * 32 * N);
    float *res = (float *)gd.get(4 * 2 * 32 * N);
    const Geo gp{32, 4, (int)((N + 127) / 128), 0, (int)N};
    size_t wpn = 0;
    for (int l = 1; l <= 3; ++l) wpn = std::max(wpn, wgrad_partial_floats(g, l));
    float *wpart = (float *)gd.get(4 * wpn), *cpart = (float *)gd.get(4 * colsum_partial_floats(gp, 32));
    float *gw = (float *)gd.get(sizeof(float) * NW);
    if (!wd || !ind || (need_aux && !auxd) || !in_cl || !in_cm || !aux_cm || !f1 || !b1 || !b2 || !res || !wpart ||
        !cpart || !gw)
        return tfail(err, HSLB_ENOMEM, "operation buffers");
    T_TRY(hipMemcpyAsync(wd, w, sizeof(float) * NW, hipMemcpyHostToDevice, s));
    T_TRY(pk.build(s, wd));
    T_TRY(hipMemcpyAsync(ind, in, sizeof(float) * c_in * N, hipMemcpyHostToDevice, s));
    if (need_aux) T_TRY(hipMemcpyAsync(auxd, aux, sizeof(float) * c_aux * N, hipMemcpyHostToDevice, s));
    FwdArgs a{};
    a.g = g;
    size_t nout = 0;
    switch (op) {
    case HSLB_CNN_FWD1:
    case HSLB_CNN_FWD2: {
        const bool l1 = op == HSLB_CNN_FWD1;
        T_TRY(launch_cm_to_bf16(s, ind, l1 ? 1 : 32, l1 ? 1 : 32, (int)N, in_cl, nullptr));
        a.in = in_cl;
        a.wp = pk.p[l1 ? PK_F1 : PK_F2];
        a.bias = wd + (l1 ? OB1 : OB2);
        a.out_cl = b1;
        a.out_f32 = f1;
        T_TRY(launch_conv_fwd(s, l1 ? 1 : 32, 32, EPI_GELU, a));
        T_TRY(launch_cl_f32_to_cm(s, f1, 32, (int)N, res));
        T_TRY(launch_cl_bf16_to_cm(s, b1, 32, (int)N, res + 32 * N));
        nout = 64 * N;
        break;
    }
    case HSLB_CNN_FWD3:
        T_TRY(launch_cm_to_bf16(s, ind, 32, 32, (int)N, in_cl, nullptr));
        a.in = in_cl;
        a.wp = pk.p[PK_F3];
        a.bias = wd + OB3;
        a.out_f32 = res;
        T_TRY(launch_conv_fwd(s, 32, 3, EPI_OUT, a));
        nout = 3 * N;
        break;
    case HSLB_CNN_DX3:
    case HSLB_CNN_DX2: {
        const bool l3 = op == HSLB_CNN_DX3;
        T_TRY(launch_cm_to_bf16(s, ind, l3 ? 3 : 32, l3 ? 4 : 32, (int)N, in_cl, nullptr));
        // the saved pre-activation, channel-last FP32
        float *zcl = (float *)gd.get(4 * 32 * N);
        if (!zcl) return tfail(err, HSLB_ENOMEM, "operation buffers");
        T_TRY(launch_cl_f32_to_cm(s, auxd, (int)N, 32, zcl));  // [32][N] -> [N][32]
        a.in = in_cl;
        a.wp = pk.p[l3 ? PK_D3 : PK_D2];
        a.zsave = zcl;
        a.out_f32 = f1;
        a.out_cl = b1;
        T_TRY(launch_conv_fwd(s, l3 ? 4 : 32, 32, EPI_DGELU, a));
        T_TRY(launch_cl_f32_to_cm(s, f1, 32, (int)N, res));
        T_TRY(launch_cl_bf16_to_cm(s, b1, 32, (int)N, res + 32 * N));
        nout = 64 * N;
        break;
    }
    default: {  // weight gradients
        const int layer = op == HSLB_CNN_DW1 ? 1 : (op == HSLB_CNN_DW2 ? 2 : 3);
        T_TRY(launch_cm_to_bf16(s, ind, c_in, c_in, (int)N, nullptr, in_cm));
        T_TRY(launch_cm_to_bf16(s, auxd, c_aux, c_aux, (int)N, nullptr, aux_cm));
        const int ow = layer == 1 ? OW1 : (layer == 2 ? OW2 : OW3);
        const int ob = layer == 1 ? OB1 : (layer == 2 ? OB2 : OB3);
        T_TRY(launch_wgrad(s, layer, g, in_cm, aux_cm, wpart, gw + ow));
        T_TRY(launch_colsum(s, g, c_aux, aux_cm, cpart, gw + ob));
        const size_t nwl = (size_t)(ob - ow);
        T_TRY(hipMemcpyAsync(out, gw + ow, sizeof(float) * (nwl + c_aux), hipMemcpyDeviceToHost, s));
        T_TRY(hipStreamSynchronize(s));
        return HSLB_OK;
    }
    }
    T_TRY(hipMemcpyAsync(out, res, sizeof(float) * nout, hipMemcpyDeviceToHost, s));
    T_TRY(hipStreamSynchronize(s));
    return HSLB_OK;
}

}  // extern "C"

// ------------------------------------------------ training from snapshot files

namespace {

constexpr char kSnapMagic[8] = {'H', 'S', 'L', 'B', 'S', 'N', 'P', '1'};

struct SnapHeader {
    int32_t nx, ny, nz, wall_lo, wall_hi, sigma;
};

// splitmix64 (Steele, Lea and Flood, 2014): the generator of the training
// order.
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

struct FileCloser {
    FILE *f;
    ~FileCloser()
    {
        if (f) std::fclose(f);
    }
};

int read_snap_header(const std::string &path, SnapHeader &h, std::string &err)
{
    FileCloser fc{std::fopen(path.c_str(), "rb")};
    if (!fc.f) return tfail(err, HSLB_EINVAL, "cannot open %s", path.c_str());
    char m[8];
    if (std::fread(m, 1, 8, fc.f) != 8 || std::memcmp(m, kSnapMagic, 8) != 0 || std::fread(&h, sizeof(h), 1, fc.f) != 1)
        return tfail(err, HSLB_EINVAL, "%s is not a snapshot file", path.c_str());
    if (!geo_ok(h.nx, h.ny, h.nz) || h.wall_lo < 0 || h.wall_hi < 0 || h.wall_lo + h.wall_hi >= h.nz ||
        ((h.wall_lo == 0) != (h.wall_hi == 0)) || (int64_t)h.nx * h.ny * h.nz >= ((int64_t)1 << 26))
        return tfail(err, HSLB_EINVAL, "%s: bad geometry", path.c_str());
    std::fseek(fc.f, 0, SEEK_END);
    const long want = 8 + (long)sizeof(h) + 14L * h.nx * h.ny * h.nz;
    if (std::ftell(fc.f) != want) return tfail(err, HSLB_EINVAL, "%s: wrong size", path.c_str());
    return HSLB_OK;
}

}  // namespace

// Adds the snapshot of file `path` (header already checked) to the store.
static int trainer_add_file(hslb_trainer *tr, const std::string &path, const SnapHeader &h)
{
    std::string &err = tr->err;
    Snapshot sn{};
    sn.g = Geo{h.nx, h.ny, h.nz, h.wall_lo == 0 ? 1 : 0, h.nx * h.ny * h.nz};
    sn.wall_lo = h.wall_lo;
    sn.wall_hi = h.wall_hi;
    const size_t N = (size_t)sn.g.N;
    int rc = tr->reserve(N, sn);
    if (rc) return rc;
    std::vector<char> buf(14 * N);
    FileCloser fc{std::fopen(path.c_str(), "rb")};
    if (!fc.f || std::fseek(fc.f, 8 + (long)sizeof(SnapHeader), SEEK_SET) != 0 ||
        std::fread(buf.data(), 1, buf.size(), fc.f) != buf.size())
        return tfail(err, HSLB_EINVAL, "cannot read %s", path.c_str());
    T_TRY(hipMemcpy(tr->arena + sn.x_off, buf.data(), 2 * N, hipMemcpyHostToDevice));
    T_TRY(hipMemcpy(tr->arena + sn.t_off, buf.data() + 2 * N, 12 * N, hipMemcpyHostToDevice));
    tr->snaps.push_back(sn);
    return HSLB_OK;
}

extern "C" {

int hslb_surrogate_save_snapshot(hslb_ctx *ctx, const char *path)
{
    if (!ctx) return HSLB_EINVAL;
    std::string err;
    if (!path) return context_fail(ctx, HSLB_EINVAL, "null path");
    Geo g{};
    int wl = 0, wh = 0, sig = 0;
    int rc = context_training_pair(ctx, nullptr, nullptr, &g, &wl, &wh, &sig, &err);  // geometry only
    if (rc) return context_fail(ctx, rc, err);
    const size_t N = (size_t)g.N;
    void *d = nullptr;
    if (hipMalloc(&d, 14 * N) != hipSuccess) return context_fail(ctx, HSLB_ENOMEM, "snapshot staging buffer");
    std::vector<char> host(14 * N);
    rc = context_training_pair(ctx, (uint16_t *)d, (float *)((char *)d + 2 * N), &g, &wl, &wh, &sig, &err);
    if (!rc && hipMemcpy(host.data(), d, 14 * N, hipMemcpyDeviceToHost) != hipSuccess) {
        rc = HSLB_EDEVICE;
        err = "snapshot copy to the host";
    }
    (void)hipFree(d);
    if (rc) return context_fail(ctx, rc, err);
    const SnapHeader h{g.nx, g.ny, g.nz, wl, wh, sig};
    FileCloser fc{std::fopen(path, "wb")};
    if (!fc.f || std::fwrite(kSnapMagic, 1, 8, fc.f) != 8 || std::fwrite(&h, sizeof(h), 1, fc.f) != 1 ||
        std::fwrite(host.data(), 1, host.size(), fc.f) != host.size())
        return context_fail(ctx, HSLB_EINVAL, std::string("cannot write ") + path);
    return HSLB_OK;
}

int hslb_surrogate_train(hslb_ctx *ctx, const char *snapshot_dir, int32_t epochs, double lr, double *final_loss)
{
    if (!ctx) return HSLB_EINVAL;
    std::string err;
    if (!snapshot_dir) return context_fail(ctx, HSLB_EINVAL, "null directory");
    if (epochs < 1) return context_fail(ctx, HSLB_EINVAL, "epochs must be >= 1");
    if (!(lr > 0.0) || !std::isfinite(lr)) return context_fail(ctx, HSLB_EINVAL, "learning rate must be > 0");
    std::vector<float> w(NW);
    int rc = hslb_surrogate_get_weights(ctx, w.data(), NW);  // also rejects a context without weights
    if (rc) return rc;
    std::vector<std::string> files;
    if (DIR *dd = opendir(snapshot_dir)) {
        while (dirent *e = readdir(dd)) {
            const std::string nm = e->d_name;
            if (nm.size() > 6 && nm.compare(nm.size() - 6, 6, ".hsnap") == 0)
                files.push_back(std::string(snapshot_dir) + "/" + nm);
        }
        closedir(dd);
    } else {
        return context_fail(ctx, HSLB_EINVAL, std::string("cannot open directory ") + snapshot_dir);
    }
    if (files.empty()) return context_fail(ctx, HSLB_EINVAL, std::string("no *.hsnap files in ") + snapshot_dir);
    std::sort(files.begin(), files.end());
    std::vector<SnapHeader> hd(files.size());
    int64_t total = 0, largest = 0;
    for (size_t k = 0; k < files.size(); ++k) {
        if ((rc = read_snap_header(files[k], hd[k], err))) return context_fail(ctx, rc, err);
        const int64_t N = (int64_t)hd[k].nx * hd[k].ny * hd[k].nz;
        total += N;
        largest = std::max(largest, N);
    }
    hslb_trainer *tr = nullptr;
    if ((rc = hslb_trainer_create(total, largest, &tr))) return context_fail(ctx, rc, hslb_trainer_last_error(nullptr));
    struct Owner {
        hslb_trainer *t;
        ~Owner() { hslb_trainer_destroy(t); }
    } own{tr};
    for (size_t k = 0; k < files.size(); ++k)
        if ((rc = trainer_add_file(tr, files[k], hd[k]))) return context_fail(ctx, rc, tr->err);
    if ((rc = hslb_trainer_set_weights(tr, w.data(), NW))) return context_fail(ctx, rc, tr->err);
    const int32_t cnt = (int32_t)files.size();
    std::vector<int32_t> order(cnt);
    double L = 0.0;
    for (int32_t ep = 0; ep < epochs; ++ep) {
        for (int32_t i = 0; i < cnt; ++i) order[i] = i;
        uint64_t st = 0x48534c42ull + (uint64_t)ep;
        for (int32_t i = cnt - 1; i >= 1; --i) {
            const int32_t j = (int32_t)(splitmix64(st) % (uint64_t)(i + 1));
            std::swap(order[i], order[j]);
        }
        if ((rc = hslb_trainer_train(tr, order.data(), cnt, lr * std::ldexp(1.0, -ep), &L)))
            return context_fail(ctx, rc, tr->err);
    }
    if ((rc = hslb_trainer_get_weights(tr, w.data(), NW))) return context_fail(ctx, rc, tr->err);
    if ((rc = hslb_surrogate_set_weights(ctx, w.data(), NW))) return rc;
    if (final_loss) *final_loss = L;
    return HSLB_OK;
}

}  // extern "C"
