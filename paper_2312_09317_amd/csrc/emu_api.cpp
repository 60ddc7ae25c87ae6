// Host side of the emulator calls declared in include/emu.h: workspace
// carving, the layer sequence of the forward and backward passes, and Adam's
// step bookkeeping.  Every arithmetic step runs in the kernels of
// emu_kernels.hip.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/emu.h"
#include "cpm_internal.hpp"
#include "emu_internal.hpp"

using namespace cpm::emu;

namespace {

constexpr int kMaxBatch = 1 << 20;

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t pad_rows(int64_t n) { return (n + kRows - 1) / kRows * kRows; }

struct EmuLayout {
    size_t params, grad, m, v, norm, loss, loss_rows;
    size_t w1, w2, w2t, w3, w3t, w4, w4t;
    size_t x, xt, z[3], a[3], at[3], y, dz4, dz4t, dza, dzat, dzb, dzbt, part;
    size_t total;
};

EmuLayout layout_for(int64_t max_batch)
{
    const int64_t np = pad_rows(max_batch);
    const int64_t splits = (np + kSplitK - 1) / kSplitK;
    EmuLayout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    l.params = take(kParams * 4);
    l.grad = take(kParams * 4);
    l.m = take(kParams * 4);
    l.v = take(kParams * 4);
    l.norm = take(EMU_NORM * 4);
    l.loss = take(4);
    l.loss_rows = take(np * 4);
    l.w1 = take((size_t)kHidden * kInPad * 2);
    l.w2 = take((size_t)kHidden * kHidden * 2);
    l.w2t = take((size_t)kHidden * kHidden * 2);
    l.w3 = take((size_t)kHidden * kHidden * 2);
    l.w3t = take((size_t)kHidden * kHidden * 2);
    l.w4 = take((size_t)kOutPad * kHidden * 2);
    l.w4t = take((size_t)kHidden * kOutPad * 2);
    l.x = take((size_t)np * kInPad * 2);
    l.xt = take((size_t)kOutPad * np * 2);  // 64 rows: the N of the first weight-gradient product
    for (int i = 0; i < 3; ++i) {
        l.z[i] = take((size_t)np * kHidden * 4);
        l.a[i] = take((size_t)np * kHidden * 2);
        l.at[i] = take((size_t)np * kHidden * 2);
    }
    l.y = take((size_t)np * kOut * 4);
    l.dz4 = take((size_t)np * kOutPad * 2);
    l.dz4t = take((size_t)np * kOutPad * 2);
    l.dza = take((size_t)np * kHidden * 2);
    l.dzat = take((size_t)np * kHidden * 2);
    l.dzb = take((size_t)np * kHidden * 2);
    l.dzbt = take((size_t)np * kHidden * 2);
    l.part = take((size_t)splits * kHidden * kHidden * 4);
    l.total = off;
    return l;
}

int fail(int code, const std::string &msg) { return cpm::report_error(code, msg.c_str()); }

int device_fail(hipError_t e, const char *where)
{
    return fail(CPM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

struct emu_handle {
    int32_t max_batch = 0;
    int64_t steps = 0;
    char *base = nullptr;
    EmuLayout l{};
    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
    float *params() const { return at<float>(l.params); }
    float *grad() const { return at<float>(l.grad); }
    float *norm() const { return at<float>(l.norm); }
};

namespace {

AdamSeg segment(const emu_handle *h, int s)
{
    AdamSeg g{};
    const int64_t begins[2 * kLayers] = {kW1, kB1, kW2, kB2, kW3, kB3, kW4, kB4};
    g.begin = begins[s];
    if (s & 1) {  // bias: no bf16 copies
        g.rows = 1;
        g.cols = s == 7 ? kOut : kHidden;
        return g;
    }
    switch (s / 2) {
    case 0:
        g.rows = kHidden, g.cols = kIn;
        g.w16 = h->at<uint16_t>(h->l.w1), g.ld16 = kInPad;
        break;
    case 1:
        g.rows = kHidden, g.cols = kHidden;
        g.w16 = h->at<uint16_t>(h->l.w2), g.ld16 = kHidden;
        g.w16_t = h->at<uint16_t>(h->l.w2t), g.ldt16 = kHidden;
        break;
    case 2:
        g.rows = kHidden, g.cols = kHidden;
        g.w16 = h->at<uint16_t>(h->l.w3), g.ld16 = kHidden;
        g.w16_t = h->at<uint16_t>(h->l.w3t), g.ldt16 = kHidden;
        break;
    default:
        g.rows = kOut, g.cols = kHidden;
        g.w16 = h->at<uint16_t>(h->l.w4), g.ld16 = kHidden;
        g.w16_t = h->at<uint16_t>(h->l.w4t), g.ldt16 = kOutPad;
        break;
    }
    return g;
}

GemmArgs gemm(const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N, int K)
{
    GemmArgs g{};
    g.A = A, g.lda = lda, g.B = B, g.ldb = ldb;
    g.M = M, g.N = N, g.K = K, g.k_chunk = K;
    g.m_store = M, g.n_store = N;
    return g;
}

int check_batch(const emu_handle *h, int32_t n)
{
    if (!h) return fail(CPM_EINVAL, "null handle");
    if (n < 1 || n > h->max_batch)
        return fail(CPM_EINVAL, "batch of " + std::to_string(n) + " points outside [1, " +
                                    std::to_string(h->max_batch) + "]");
    return CPM_OK;
}

// Forward pass over n points; keep = store what the backward pass reads
// (pre-activations and transposed activations).  Leaves the normalised
// outputs in y.
hipError_t forward(emu_handle *h, const float *d_x, int n, bool keep, hipStream_t st)
{
    const EmuLayout &l = h->l;
    const int np = (int)pad_rows(n);
    hipError_t e;
    uint16_t *x = h->at<uint16_t>(l.x);
    if ((e = launch_input(d_x, n, np, h->norm(), x, keep ? h->at<uint16_t>(l.xt) : nullptr, np, st)) != hipSuccess)
        return e;
    const uint16_t *in = x;
    int ld_in = kInPad, k_in = kInPad;
    const size_t w[3] = {l.w1, l.w2, l.w3};
    const int64_t b[3] = {kB1, kB2, kB3};
    for (int i = 0; i < 3; ++i) {
        GemmArgs g = gemm(in, ld_in, h->at<uint16_t>(w[i]), k_in, np, kHidden, k_in);
        g.bias = h->params() + b[i];
        g.C = keep ? h->at<float>(l.z[i]) : nullptr;
        g.ldc = kHidden;
        g.out = h->at<uint16_t>(l.a[i]);
        g.ldo = kHidden;
        g.out_t = keep ? h->at<uint16_t>(l.at[i]) : nullptr;
        g.ldot = np;
        if ((e = launch_gemm(kEpiBiasGelu, g, st)) != hipSuccess) return e;
        in = g.out;
        ld_in = k_in = kHidden;
    }
    GemmArgs g = gemm(in, kHidden, h->at<uint16_t>(l.w4), kHidden, np, kOutPad, kHidden);
    g.bias = h->params() + kB4;
    g.C = h->at<float>(l.y);
    g.ldc = kOut;
    g.n_store = kOut;
    return launch_gemm(kEpiBias, g, st);
}

// dW = dZ^T . A_prev over the batch (K = np), split over K in chunks of
// kSplitK with a fixed-order reduction; rows m < m_store and columns
// n < n_store land in out (pitch ldo).
hipError_t weight_grad(emu_handle *h, const uint16_t *dz_t, int M, const uint16_t *a_t, int N, int np, int m_store,
                       int n_store, float *out, int ldo, hipStream_t st)
{
    GemmArgs g = gemm(dz_t, np, a_t, np, M, N, np);
    g.m_store = m_store, g.n_store = n_store;
    const int splits = (np + kSplitK - 1) / kSplitK;
    if (splits == 1) {
        g.C = out, g.ldc = ldo;
        return launch_gemm(kEpiPlain, g, st);
    }
    g.k_chunk = kSplitK;
    g.C = h->at<float>(h->l.part);
    g.c_split = (int64_t)M * N;
    g.ldc = N;
    hipError_t e = launch_gemm(kEpiPlain, g, st);
    if (e != hipSuccess) return e;
    return launch_split_reduce(g.C, splits, g.c_split, M, N, m_store, n_store, out, ldo, st);
}

// dL/dz of a hidden layer: (dZ_next . W_next) * GELU'(z).
hipError_t hidden_grad(emu_handle *h, const uint16_t *dz_next, int ld_next, const uint16_t *w_t, int k, size_t z,
                       uint16_t *dz, uint16_t *dz_t, int np, hipStream_t st)
{
    GemmArgs g = gemm(dz_next, ld_next, w_t, k, np, kHidden, k);
    g.Z = h->at<float>(z), g.ldz = kHidden;
    g.out = dz, g.ldo = kHidden;
    g.out_t = dz_t, g.ldot = np;
    return launch_gemm(kEpiGeluGrad, g, st);
}

hipError_t backward(emu_handle *h, const float *d_t, int n, hipStream_t st)
{
    const EmuLayout &l = h->l;
    const int np = (int)pad_rows(n);
    float *gr = h->grad();
    uint16_t *dz4 = h->at<uint16_t>(l.dz4), *dz4t = h->at<uint16_t>(l.dz4t);
    uint16_t *dza = h->at<uint16_t>(l.dza), *dzat = h->at<uint16_t>(l.dzat);
    uint16_t *dzb = h->at<uint16_t>(l.dzb), *dzbt = h->at<uint16_t>(l.dzbt);
    hipError_t e;
    if ((e = launch_loss(h->at<float>(l.y), d_t, n, np, h->norm(), dz4, dz4t, h->at<float>(l.loss_rows), st)) !=
        hipSuccess)
        return e;
    if ((e = launch_loss_sum(h->at<float>(l.loss_rows), n, h->at<float>(l.loss), st)) != hipSuccess) return e;
    // layer 4
    if ((e = weight_grad(h, dz4t, kOutPad, h->at<uint16_t>(l.at[2]), kHidden, np, kOut, kHidden, gr + kW4, kHidden,
                         st)) != hipSuccess)
        return e;
    if ((e = launch_rowsum(dz4t, kOut, np, gr + kB4, st)) != hipSuccess) return e;
    // layer 3
    if ((e = hidden_grad(h, dz4, kOutPad, h->at<uint16_t>(l.w4t), kOutPad, l.z[2], dza, dzat, np, st)) != hipSuccess)
        return e;
    if ((e = weight_grad(h, dzat, kHidden, h->at<uint16_t>(l.at[1]), kHidden, np, kHidden, kHidden, gr + kW3, kHidden,
                         st)) != hipSuccess)
        return e;
    if ((e = launch_rowsum(dzat, kHidden, np, gr + kB3, st)) != hipSuccess) return e;
    // layer 2
    if ((e = hidden_grad(h, dza, kHidden, h->at<uint16_t>(l.w3t), kHidden, l.z[1], dzb, dzbt, np, st)) != hipSuccess)
        return e;
    if ((e = weight_grad(h, dzbt, kHidden, h->at<uint16_t>(l.at[0]), kHidden, np, kHidden, kHidden, gr + kW2, kHidden,
                         st)) != hipSuccess)
        return e;
    if ((e = launch_rowsum(dzbt, kHidden, np, gr + kB2, st)) != hipSuccess) return e;
    // layer 1
    if ((e = hidden_grad(h, dzb, kHidden, h->at<uint16_t>(l.w2t), kHidden, l.z[0], dza, dzat, np, st)) != hipSuccess)
        return e;
    if ((e = weight_grad(h, dzat, kHidden, h->at<uint16_t>(l.xt), kOutPad, np, kHidden, kIn, gr + kW1, kIn, st)) !=
        hipSuccess)
        return e;
    return launch_rowsum(dzat, kHidden, np, gr + kB1, st);
}

hipError_t refresh_copies(emu_handle *h, hipStream_t st)
{
    for (int s = 0; s < 2 * kLayers; s += 2) {
        hipError_t e = launch_cast(segment(h, s), h->params(), st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int emu_param_count(int64_t *count)
{
    if (!count) return fail(CPM_EINVAL, "null count");
    *count = kParams;
    return CPM_OK;
}

int emu_workspace_bytes(int32_t max_batch, size_t *bytes)
{
    if (!bytes) return fail(CPM_EINVAL, "null bytes");
    if (max_batch < 1 || max_batch > kMaxBatch) return fail(CPM_EINVAL, "max_batch outside [1, 2^20]");
    *bytes = layout_for(max_batch).total;
    return CPM_OK;
}

int emu_init(int32_t max_batch, void *d_workspace, size_t workspace_bytes, void *stream, emu_handle **out)
{
    if (!out || !d_workspace) return fail(CPM_EINVAL, "null pointer");
    *out = nullptr;
    if (max_batch < 1 || max_batch > kMaxBatch) return fail(CPM_EINVAL, "max_batch outside [1, 2^20]");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return fail(CPM_EINVAL, "workspace not 256-byte aligned");
    const EmuLayout l = layout_for(max_batch);
    if (workspace_bytes < l.total)
        return fail(CPM_ENOMEM, "workspace of " + std::to_string(workspace_bytes) + " bytes, need " +
                                    std::to_string(l.total));
    emu_handle *h = new (std::nothrow) emu_handle;
    if (!h) return fail(CPM_ENOMEM, "host allocation");
    h->max_batch = max_batch;
    h->base = static_cast<char *>(d_workspace);
    h->l = l;
    hipStream_t st = as_stream(stream);
    hipError_t e;
    // parameters, Adam state and every bf16 copy (with its zero padding) start at zero
    if ((e = launch_fill_f32(h->params(), 0.f, (int64_t)(l.x - l.params) / 4, st)) != hipSuccess) {
        delete h;
        return device_fail(e, "emu_init");
    }
    float *norm = h->norm();
    if ((e = launch_fill_f32(norm + kIn, 1.f, kIn, st)) != hipSuccess ||
        (e = launch_fill_f32(norm + 2 * kIn + kOut, 1.f, kOut, st)) != hipSuccess) {
        delete h;
        return device_fail(e, "emu_init");
    }
    *out = h;
    return CPM_OK;
}

int emu_set_params(emu_handle *h, const float *d_params, void *stream)
{
    if (!h || !d_params) return fail(CPM_EINVAL, "null pointer");
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(h->params(), d_params, kParams * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = launch_fill_f32(h->at<float>(h->l.m), 0.f, kParams, st);
    if (e == hipSuccess) e = launch_fill_f32(h->at<float>(h->l.v), 0.f, kParams, st);
    if (e == hipSuccess) e = refresh_copies(h, st);
    if (e != hipSuccess) return device_fail(e, "emu_set_params");
    h->steps = 0;
    return CPM_OK;
}

int emu_get_params(emu_handle *h, float *d_params, void *stream)
{
    if (!h || !d_params) return fail(CPM_EINVAL, "null pointer");
    hipError_t e = hipMemcpyAsync(d_params, h->params(), kParams * 4, hipMemcpyDeviceToDevice, as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "emu_get_params");
}

int emu_set_norm(emu_handle *h, const float *d_norm, void *stream)
{
    if (!h || !d_norm) return fail(CPM_EINVAL, "null pointer");
    hipError_t e = hipMemcpyAsync(h->norm(), d_norm, EMU_NORM * 4, hipMemcpyDeviceToDevice, as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "emu_set_norm");
}

int emu_get_norm(emu_handle *h, float *d_norm, void *stream)
{
    if (!h || !d_norm) return fail(CPM_EINVAL, "null pointer");
    hipError_t e = hipMemcpyAsync(d_norm, h->norm(), EMU_NORM * 4, hipMemcpyDeviceToDevice, as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "emu_get_norm");
}

int emu_fit_norm(emu_handle *h, const float *d_x, const float *d_targets, int32_t n, int32_t log_mask, void *stream)
{
    if (!h || !d_x || !d_targets) return fail(CPM_EINVAL, "null pointer");
    if (n < 1) return fail(CPM_EINVAL, "empty data set");
    if (log_mask < 0 || log_mask > 0xFF) return fail(CPM_EINVAL, "log_mask has bits beyond the 8 outputs");
    hipError_t e = launch_fit_norm(d_x, d_targets, n, log_mask, h->norm(), as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "emu_fit_norm");
}

int emu_forward(emu_handle *h, const float *d_x, int32_t n, float *d_y, void *stream)
{
    int rc = check_batch(h, n);
    if (rc != CPM_OK) return rc;
    if (!d_x || !d_y) return fail(CPM_EINVAL, "null pointer");
    hipStream_t st = as_stream(stream);
    hipError_t e = forward(h, d_x, n, false, st);
    if (e == hipSuccess) e = launch_output(h->at<float>(h->l.y), n, h->norm(), d_y, st);
    return e == hipSuccess ? CPM_OK : device_fail(e, "emu_forward");
}

int emu_grads(emu_handle *h, const float *d_x, const float *d_targets, int32_t n, float *d_grad, float *d_loss,
              void *stream)
{
    int rc = check_batch(h, n);
    if (rc != CPM_OK) return rc;
    if (!d_x || !d_targets) return fail(CPM_EINVAL, "null pointer");
    hipStream_t st = as_stream(stream);
    hipError_t e = forward(h, d_x, n, true, st);
    if (e == hipSuccess) e = backward(h, d_targets, n, st);
    if (e == hipSuccess && d_grad) e = hipMemcpyAsync(d_grad, h->grad(), kParams * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && d_loss)
        e = hipMemcpyAsync(d_loss, h->at<float>(h->l.loss), 4, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? CPM_OK : device_fail(e, "emu_grads");
}

int emu_adam(emu_handle *h, const float *d_grad, float lr, void *stream)
{
    if (!h) return fail(CPM_EINVAL, "null handle");
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(CPM_EINVAL, "learning rate must be positive and finite");
    AdamArgs a{};
    a.param = h->params();
    a.m = h->at<float>(h->l.m);
    a.v = h->at<float>(h->l.v);
    a.grad = d_grad ? d_grad : h->grad();
    a.n = kParams;
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.one_minus_beta1 = 0.1f;
    a.one_minus_beta2 = 0.001f;
    a.eps = 1e-8f;
    const int64_t t = h->steps + 1;
    a.c1 = (float)(1.0 - std::pow(0.9, (double)t));
    a.c2 = (float)(1.0 - std::pow(0.999, (double)t));
    for (int s = 0; s < 2 * kLayers; ++s) a.seg[s] = segment(h, s);
    hipError_t e = launch_adam(a, as_stream(stream));
    if (e != hipSuccess) return device_fail(e, "emu_adam");
    h->steps = t;
    return CPM_OK;
}

int emu_train_step(emu_handle *h, const float *d_x, const float *d_targets, int32_t n, float lr, float *d_loss,
                   void *stream)
{
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(CPM_EINVAL, "learning rate must be positive and finite");
    int rc = emu_grads(h, d_x, d_targets, n, nullptr, d_loss, stream);
    if (rc != CPM_OK) return rc;
    return emu_adam(h, nullptr, lr, stream);
}

int emu_step_count(emu_handle *h, int64_t *steps)
{
    if (!h || !steps) return fail(CPM_EINVAL, "null pointer");
    *steps = h->steps;
    return CPM_OK;
}

int emu_destroy(emu_handle *h)
{
    delete h;
    return CPM_OK;
}

}  // extern "C"
