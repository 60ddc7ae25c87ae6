// Cell-level summary statistics of batched runs: per-cell samples (volume,
// surface, centroid) taken every few MCS, reduced per lattice to the means
// and variances of volume, surface, speed and persistence time.  FP64, with
// floating-point contraction off so that every per-cell quantity is
// rounded exactly as written.
//
// Speed and directional persistence are the motility read-outs of the paper
// (Results, Fig. 5B: directional autocorrelation; the tissue-model sections:
// cell speeds); the paper gives no formula, the definitions follow.
//   speed:       |d_k| / interval, d_k the minimum-image centroid
//                displacement between consecutive samples (cell alive at both)
//   persistence: first lag where A(tau) = mean_k u_k . u_{k+tau} of the unit
//                displacements drops below 1/e, linearly interpolated between
//                the lags, in MCS; the longest defined lag if it never does
#include "cpm_internal.hpp"

#pragma clang fp contract(off)

namespace cpm {
namespace {

constexpr int kRec = 5;  // V, S, x, y, z

__device__ __forceinline__ int find_lattice(const int64_t *off, int n, int64_t j)
{
    int lo = 0, hi = n;  // off[lo] <= j < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (off[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

// One record per label: (V, S, centroid position in [0, L) per axis).
__global__ void sample_kernel(const StatsTables t, const int32_t *vol, const int32_t *surf, const int64_t *csum,
                              double *samples, int k, int n_samples)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= t.label_off[t.n]) return;
    const int i = find_lattice(t.label_off, t.n, j);
    const int64_t c = j - t.label_off[i];
    const int64_t labels = t.label_off[i + 1] - t.label_off[i];
    double *rec = samples + (t.label_off[i] * n_samples + (int64_t)k * labels + c) * kRec;
    const int32_t v = vol[j];
    rec[0] = (double)v;
    rec[1] = (double)surf[j];
    for (int d = 0; d < 3; ++d) {
        double x = 0.0;
        if (d < t.ndim && v > 0) {
            const double L = (double)t.dims[3 * i + d];
            x = fmod((double)csum[j * t.ndim + d] / (double)v, L);
            if (x < 0.0) x += L;
        }
        rec[2 + d] = x;
    }
}

__device__ double block_sum(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Displacement of cell c between samples k and k+1 (minimum image); false if
// the cell is dead at either sample.
__device__ __forceinline__ bool displacement(const double *base, int64_t labels, int ndim, const double *L, int k,
                                             int64_t c, double *d)
{
    const double *a = base + ((int64_t)k * labels + c) * kRec;
    const double *b = base + ((int64_t)(k + 1) * labels + c) * kRec;
    if (!(a[0] > 0.0) || !(b[0] > 0.0)) return false;
    for (int e = 0; e < ndim; ++e) {
        const double x = b[2 + e] - a[2 + e];
        d[e] = x - L[e] * rint(x / L[e]);
    }
    return true;
}

// One workgroup per lattice.
__global__ void __launch_bounds__(256) summary_kernel(const StatsTables t, const double *samples, int n_samples,
                                                      double interval, double *out)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t labels = t.label_off[i + 1] - t.label_off[i];
    const double *base = samples + t.label_off[i] * n_samples * kRec;
    const int ndim = t.ndim;
    double L[3];
    for (int d = 0; d < 3; ++d) L[d] = (double)t.dims[3 * i + d];
    const int K = n_samples;
    const double inv_e = exp(-1.0);

    double n_vs = 0, sv = 0, svv = 0, ss = 0, sss = 0;
    double n_sp = 0, ssp = 0, sspp = 0;
    double n_pe = 0, spe = 0, spee = 0;
    for (int64_t c = 1 + tid; c < labels; c += blockDim.x) {
        for (int k = 0; k < K; ++k) {
            const double *r = base + ((int64_t)k * labels + c) * kRec;
            if (r[0] > 0.0) {
                n_vs += 1.0;
                sv += r[0];
                svv += r[0] * r[0];
                ss += r[1];
                sss += r[1] * r[1];
            }
        }
        // speeds and persistence of cell c
        bool any_lag = false, done = false;
        double a_prev = 1.0, p = 0.0;
        int last = 0;
        for (int k = 0; k + 1 < K; ++k) {
            double d[3] = {0, 0, 0};
            if (displacement(base, labels, ndim, L, k, c, d)) {
                double n2 = 0.0;
                for (int e = 0; e < ndim; ++e) n2 = n2 + d[e] * d[e];
                const double sp = sqrt(n2) / interval;
                n_sp += 1.0;
                ssp += sp;
                sspp += sp * sp;
            }
        }
        const int m = K - 1;  // displacement steps
        for (int tau = 1; tau < m && !done; ++tau) {
            double acc = 0.0;
            int cnt = 0;
            for (int k = 0; k + tau < m; ++k) {
                double u[3] = {0, 0, 0}, w[3] = {0, 0, 0};
                if (!displacement(base, labels, ndim, L, k, c, u)) continue;
                if (!displacement(base, labels, ndim, L, k + tau, c, w)) continue;
                double nu = 0.0, nw = 0.0;
                for (int e = 0; e < ndim; ++e) {
                    nu = nu + u[e] * u[e];
                    nw = nw + w[e] * w[e];
                }
                nu = sqrt(nu);
                nw = sqrt(nw);
                if (!(nu > 0.0) || !(nw > 0.0)) continue;
                double dot = 0.0;
                for (int e = 0; e < ndim; ++e) dot = dot + (u[e] / nu) * (w[e] / nw);
                acc = acc + dot;
                ++cnt;
            }
            if (cnt == 0) continue;
            any_lag = true;
            const double a = acc / (double)cnt;
            if (a < inv_e) {
                // linear between the last defined lag and this one
                p = (double)last + (double)(tau - last) * (a_prev - inv_e) / (a_prev - a);
                done = true;
            } else {
                a_prev = a;
                last = tau;
            }
        }
        if (any_lag) {
            if (!done) p = (double)last;
            const double pm = p * interval;
            n_pe += 1.0;
            spe += pm;
            spee += pm * pm;
        }
    }
    const double tot[11] = {n_vs, sv, svv, ss, sss, n_sp, ssp, sspp, n_pe, spe, spee};
    double r[11];
    for (int q = 0; q < 11; ++q) r[q] = block_sum(tot[q], red);
    if (tid == 0) {
        double *o = out + 8 * (int64_t)i;
        auto moments = [](double n, double s1, double s2, double *mv) {
            if (n > 0) {
                const double mean = s1 / n;
                mv[0] = mean;
                mv[1] = s2 / n - mean * mean;
            } else {
                mv[0] = 0.0;
                mv[1] = 0.0;
            }
        };
        moments(r[0], r[1], r[2], o);
        moments(r[0], r[3], r[4], o + 2);
        moments(r[5], r[6], r[7], o + 4);
        moments(r[8], r[9], r[10], o + 6);
    }
}

// Unit displacement of cell c over step k (false when undefined: the cell is
// dead at either sample or did not move).
__device__ __forceinline__ bool unit_step(const double *base, int64_t labels, int ndim, const double *L, int k,
                                          int64_t c, double *u)
{
    if (!displacement(base, labels, ndim, L, k, c, u)) return false;
    double n = 0.0;
    for (int e = 0; e < ndim; ++e) n = n + u[e] * u[e];
    n = sqrt(n);
    if (!(n > 0.0)) return false;
    for (int e = 0; e < ndim; ++e) u[e] = u[e] / n;
    return true;
}

// Directional autocorrelation of lattice blockIdx.x: per lag tau, the sum of
// u_k . u_{k+tau} over cells and steps with both unit steps defined, and the
// number of such pairs.  One workgroup per lattice, cells strided over its
// threads; lags one after another.
__global__ void __launch_bounds__(256) autocorr_kernel(const StatsTables t, const double *samples, int n_samples,
                                                       double *out)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t labels = t.label_off[i + 1] - t.label_off[i];
    const double *base = samples + t.label_off[i] * n_samples * kRec;
    const int ndim = t.ndim;
    double L[3];
    for (int d = 0; d < 3; ++d) L[d] = (double)t.dims[3 * i + d];
    const int m = n_samples - 1;  // steps
    for (int tau = 0; tau < m; ++tau) {
        double acc = 0.0, cnt = 0.0;
        for (int64_t c = 1 + tid; c < labels; c += blockDim.x) {
            for (int k = 0; k + tau < m; ++k) {
                double u[3] = {0, 0, 0}, w[3] = {0, 0, 0};
                if (!unit_step(base, labels, ndim, L, k, c, u)) continue;
                if (!unit_step(base, labels, ndim, L, k + tau, c, w)) continue;
                double dot = 0.0;
                for (int e = 0; e < ndim; ++e) dot = dot + u[e] * w[e];
                acc = acc + dot;
                cnt = cnt + 1.0;
            }
        }
        const double sa = block_sum(acc, red), sc = block_sum(cnt, red);
        if (tid == 0) {
            out[2 * ((int64_t)i * m + tau)] = sa;
            out[2 * ((int64_t)i * m + tau) + 1] = sc;
        }
    }
}

}  // namespace

hipError_t launch_autocorrelation(const StatsTables &t, const double *samples, int n_samples, double *out,
                                  hipStream_t stream)
{
    autocorr_kernel<<<t.n, 256, 0, stream>>>(t, samples, n_samples, out);
    return hipGetLastError();
}

hipError_t launch_sample(const StatsTables &t, const int32_t *vol, const int32_t *surf, const int64_t *csum,
                         double *samples, int k, int n_samples, hipStream_t stream)
{
    const int64_t total = t.total_labels;
    sample_kernel<<<(unsigned)((total + 255) / 256), 256, 0, stream>>>(t, vol, surf, csum, samples, k, n_samples);
    return hipGetLastError();
}

hipError_t launch_summary(const StatsTables &t, const double *samples, int n_samples, double interval, double *out,
                          hipStream_t stream)
{
    summary_kernel<<<t.n, 256, 0, stream>>>(t, samples, n_samples, interval, out);
    return hipGetLastError();
}

}  // namespace cpm
