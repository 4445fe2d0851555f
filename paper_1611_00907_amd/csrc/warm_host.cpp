// Host helpers of the learned warm start (no GPU work): the circular-cap density of
// a drop on the wall, the logarithmic phase map and its inverse, the smoothing of a
// predicted phase field and the bulk phase levels read off it.  They run per case on
// host threads (the calls hold no interpreter lock), so a batch of warm fields is
// built in parallel.
#include <algorithm>
#include <cmath>
#include <vector>

#include "lbm.h"

namespace {

// Median of v (the mean of the two middle values for an even count), as numpy's.
double median_of(std::vector<float>& v) {
    const size_t n = v.size(), h = n / 2;
    std::nth_element(v.begin(), v.begin() + h, v.end());
    const float upper = v[h];
    if (n % 2) return upper;
    const float lower = *std::max_element(v.begin(), v.begin() + h);
    return double((lower + upper) * 0.5f);
}

}  // namespace

extern "C" {

lbm_status lbm_warm_cap(int32_t nx, int32_t ny, double rho_in, double rho_out, double radius, double cx, double cy,
                        double width, double* out) {
    if (nx < 1 || ny < 1 || !out || !(width > 0) || !std::isfinite(radius + cx + cy + rho_in + rho_out))
        return LBM_EINVAL;
    const double mid = 0.5 * (rho_in + rho_out), half = 0.5 * (rho_in - rho_out), k = 2.0 / width;
    for (int32_t y = 0; y < ny; ++y) {
        const double dy = double(y) - cy;
        double* row = out + (size_t)y * nx;
        for (int32_t x = 0; x < nx; ++x) {
            const double dx = double(x) - cx;
            const double u = k * (std::sqrt(dx * dx + dy * dy) - radius);
            // tanh(u) = 1 - 2 / (exp(2 u) + 1); beyond |u| = 20 it is +-1 to double precision
            const double t = u > 20.0 ? 1.0 : (u < -20.0 ? -1.0 : 1.0 - 2.0 / (std::exp(2.0 * u) + 1.0));
            row[x] = mid - half * t;
        }
    }
    return LBM_OK;
}

lbm_status lbm_warm_phase(int64_t n, const double* rho, double rho_g, double rho_l, float* out) {
    if (n < 0 || (n && (!rho || !out)) || !(rho_g > 0) || !(rho_l > rho_g)) return LBM_EINVAL;
    const double inv = 1.0 / std::log(rho_l / rho_g);
    for (int64_t i = 0; i < n; ++i) out[i] = float(std::log(std::max(rho[i], 1e-300) / rho_g) * inv);
    return LBM_OK;
}

lbm_status lbm_warm_density(int64_t n, const float* phi, double rho_g, double rho_l, double* out) {
    if (n < 0 || (n && (!phi || !out)) || !(rho_g > 0) || !(rho_l > rho_g)) return LBM_EINVAL;
    const double l = std::log(rho_l / rho_g);
    for (int64_t i = 0; i < n; ++i) out[i] = rho_g * std::exp(double(phi[i]) * l);
    return LBM_OK;
}

lbm_status lbm_warm_smooth(int32_t nx, int32_t ny, const float* pred, float lo, float hi, float* out) {
    if (nx < 1 || ny < 1 || !pred || !out || !(lo <= hi)) return LBM_EINVAL;
    // clipped copy with one halo node: x periodic, rows clamped
    const int32_t W = nx + 2;
    std::vector<float> p((size_t)(ny + 2) * W);
    for (int32_t y = -1; y <= ny; ++y) {
        const float* src = pred + (size_t)(y < 0 ? 0 : (y >= ny ? ny - 1 : y)) * nx;
        float* dst = p.data() + (size_t)(y + 1) * W;
        for (int32_t x = 0; x < nx; ++x) dst[x + 1] = std::min(std::max(src[x], lo), hi);
        dst[0] = dst[nx];
        dst[nx + 1] = dst[1];
    }
    const float wc = 4.0f / 9.0f, wa = 1.0f / 9.0f, wd = 1.0f / 36.0f;
    for (int32_t y = 0; y < ny; ++y) {
        const float *a = p.data() + (size_t)y * W + 1, *b = a + W, *c = b + W;  // rows y - 1, y, y + 1
        float* o = out + (size_t)y * nx;
        for (int32_t x = 0; x < nx; ++x) {
            const float ax = (a[x] + c[x]) + (b[x - 1] + b[x + 1]);
            const float dg = (a[x - 1] + a[x + 1]) + (c[x - 1] + c[x + 1]);
            o[x] = wc * b[x] + wa * ax + wd * dg;
        }
    }
    return LBM_OK;
}

lbm_status lbm_warm_bulk_phases(int32_t nx, int32_t ny, const float* phi, double* ph_l, double* ph_g) {
    if (nx < 1 || ny < 1 || !phi || !ph_l || !ph_g) return LBM_EINVAL;
    const size_t n = (size_t)nx * ny;
    std::vector<int> xw(nx + 4), yw(ny + 4);  // wrapped indices of x - 2 .. x + 2, y - 2 .. y + 2
    for (int32_t k = 0; k < nx + 4; ++k) xw[k] = ((k - 2) % nx + nx) % nx;
    for (int32_t k = 0; k < ny + 4; ++k) yw[k] = ((k - 2) % ny + ny) % ny;
    std::vector<unsigned char> hi(n), row_hi(n), row_lo(n);
    for (size_t i = 0; i < n; ++i) hi[i] = phi[i] > 0.5f;
    // 5 x 5 erosions of both sides, separably, periodic in x and y
    for (int32_t y = 0; y < ny; ++y) {
        const unsigned char* h = hi.data() + (size_t)y * nx;
        for (int32_t x = 0; x < nx; ++x) {
            const int s = h[xw[x]] + h[xw[x + 1]] + h[xw[x + 2]] + h[xw[x + 3]] + h[xw[x + 4]];
            row_hi[(size_t)y * nx + x] = s == 5;
            row_lo[(size_t)y * nx + x] = s == 0;
        }
    }
    std::vector<float> liq, vap;
    liq.reserve(n);
    vap.reserve(n);
    for (int32_t y = 0; y < ny; ++y) {
        const size_t r0 = (size_t)yw[y] * nx, r1 = (size_t)yw[y + 1] * nx, r2 = (size_t)yw[y + 2] * nx,
                     r3 = (size_t)yw[y + 3] * nx, r4 = (size_t)yw[y + 4] * nx;
        for (int32_t x = 0; x < nx; ++x) {
            if (row_hi[r0 + x] & row_hi[r1 + x] & row_hi[r2 + x] & row_hi[r3 + x] & row_hi[r4 + x])
                liq.push_back(phi[(size_t)y * nx + x]);
            if (row_lo[r0 + x] & row_lo[r1 + x] & row_lo[r2 + x] & row_lo[r3 + x] & row_lo[r4 + x])
                vap.push_back(phi[(size_t)y * nx + x]);
        }
    }
    *ph_l = liq.empty() ? 1.0 : median_of(liq);
    *ph_g = vap.empty() ? 0.0 : median_of(vap);
    return LBM_OK;
}

}  // extern "C"
