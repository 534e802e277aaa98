// Orientation samplers (Sec. IV-C) for gfx950: one thread per sample, the
// geometry in FP64, the quaternion rounded to float32 at the end.
//
// Super-Fibonacci (the construction the paper adopts for the global search):
// for s = i + 1/2, r = sqrt(s/n), R = sqrt(1 - s/n), angles 2 pi frac(s/phi)
// and 2 pi frac(s/psi), phi = sqrt 2, psi the root above 1 of x^4 = x + 4;
// q = (r sin a, r cos a, R sin b, R cos b).
//
// GeoBall-SF (Alg. geoball-sf): with q = (R cos a, R sin a, r cos b, r sin b)
// the ball of radius theta around the identity is |a| <= L(r)/2,
// L(r) = 2 arccos(cos theta / R), and the uniform measure is r dr da db, so the
// radius has density r L(r) on [0, sin theta].  Its distribution function is
// tabulated on the host (uniform grid of r, cumulative trapezoid rule,
// GEOBALL_TABLE points) and inverted in the kernel by bisection and linear
// interpolation; the sample is q0 * q_local.
#include "so3_sampling.h"

#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "runtime.h"

namespace regdock {

// Radial table of the allocation-free GeoBall-SF entry point: radii, then the
// normalised distribution function, GEOBALL_TABLE doubles each (64 KiB).  Each
// device holds its own copy for the life of the process; host code reaches it
// only through the address hipGetSymbolAddress gives on that device.
static __device__ __align__(256) double scratch[2 * GEOBALL_TABLE];

namespace {

constexpr double TWO_PI = 6.283185307179586476925286766559;

double psi_constant() {
    double x = 1.5;  // Newton on x^4 - x - 4
    for (int i = 0; i < 60; ++i) x -= (x * x * x * x - x - 4.0) / (4.0 * x * x * x - 1.0);
    return x;
}

__device__ __forceinline__ double frac(double v) { return v - floor(v); }

__global__ __launch_bounds__(256) void k_super_fibonacci(int n, double inv_phi, double inv_psi, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = (double)i + 0.5;
    const double r = sqrt(s / n), R = sqrt(1.0 - s / n);
    double sa, ca, sb, cb;
    sincos(TWO_PI * frac(s * inv_phi), &sa, &ca);
    sincos(TWO_PI * frac(s * inv_psi), &sb, &cb);
    reinterpret_cast<float4*>(out)[i] = make_float4((float)(r * sa), (float)(r * ca), (float)(R * sb), (float)(R * cb));
}

__global__ __launch_bounds__(256) void k_geoball_sf(int n, double q0w, double q0x, double q0y, double q0z,
                                                    double cos_theta, double gamma, double inv_phi, double inv_psi,
                                                    const double* __restrict__ tr, const double* __restrict__ tF,
                                                    int points, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = (double)i + 0.5;
    const double u1 = frac(s / gamma), u2 = frac(s * inv_phi), u3 = frac(s * inv_psi);
    // F is strictly increasing from 0 to 1: the segment [F_lo, F_hi] holding u1
    int lo = 0, hi = points - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tF[mid] <= u1) lo = mid;
        else hi = mid;
    }
    const double t = (u1 - tF[lo]) / (tF[hi] - tF[lo]);
    const double r = tr[lo] + t * (tr[hi] - tr[lo]);
    const double R = sqrt(1.0 - r * r);
    const double L = 2.0 * acos(fmin(1.0, cos_theta / R));
    double sa, ca, sb, cb;
    sincos((u2 - 0.5) * L, &sa, &ca);
    sincos(TWO_PI * u3, &sb, &cb);
    const double w = R * ca, x = R * sa, y = r * cb, z = r * sb;
    reinterpret_cast<float4*>(out)[i] = make_float4((float)(q0w * w - q0x * x - q0y * y - q0z * z),
                                                    (float)(q0w * x + q0x * w + q0y * z - q0z * y),
                                                    (float)(q0w * y - q0x * z + q0y * w + q0z * x),
                                                    (float)(q0w * z + q0x * y - q0y * x + q0z * w));
}

// Radial distribution function of GeoBall-SF on the device, the same
// quantity the host tabulates for geoball_sf: radii on a uniform grid of
// [0, sin theta], the density r L(r) at each, its cumulative trapezoid sum in
// grid order (one thread, so the sum is in a fixed order), normalised to 1.
__global__ __launch_bounds__(256) void k_geoball_table(double* __restrict__ tab, int points, double theta) {
    double* tr = tab;
    double* tF = tab + points;
    __shared__ double total;
    const double rmax = sin(theta), ct = cos(theta);
    for (int j = threadIdx.x; j < points; j += blockDim.x) {
        const double r = rmax * (double)j / (double)(points - 1);
        const double c = ct / sqrt(1.0 - r * r);
        tr[j] = r;
        tF[j] = r * 2.0 * acos(c < 1.0 ? c : 1.0);  // density, summed below
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double prev = tF[0], acc = 0.0;
        tF[0] = 0.0;
        for (int j = 1; j < points; ++j) {
            const double d = tF[j];
            acc += 0.5 * (d + prev) * (tr[j] - tr[j - 1]);
            tF[j] = acc;
            prev = d;
        }
        total = acc;
    }
    __syncthreads();
    const double inv = total;
    for (int j = threadIdx.x; j < points; j += blockDim.x) tF[j] /= inv;
}

// device address of `scratch` on the current device, looked up once per device
hipError_t scratch_address(double** out) {
    static std::mutex mu;
    static std::map<int, double*> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = addr.emplace(dev, static_cast<double*>(ptr)).first;
    }
    *out = it->second;
    return hipSuccess;
}

}  // namespace

hipError_t geoball_sf_noalloc(int n, const double* q0, double theta, double gamma, float* out, hipStream_t s) {
    double* tab = nullptr;
    hipError_t e = scratch_address(&tab);
    if (e != hipSuccess) return e;
    const double qn = std::sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
    k_geoball_table<<<1, 256, 0, s>>>(tab, GEOBALL_TABLE, theta);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_geoball_sf<<<(n + 255) / 256, 256, 0, s>>>(n, q0[0] / qn, q0[1] / qn, q0[2] / qn, q0[3] / qn, std::cos(theta),
                                                 gamma > 0.0 ? gamma : (double)n, 1.0 / std::sqrt(2.0),
                                                 1.0 / psi_constant(), tab, tab + GEOBALL_TABLE, GEOBALL_TABLE, out);
    return hipGetLastError();
}

hipError_t super_fibonacci(int n, float* out, hipStream_t s) {
    k_super_fibonacci<<<(n + 255) / 256, 256, 0, s>>>(n, 1.0 / std::sqrt(2.0), 1.0 / psi_constant(), out);
    return hipGetLastError();
}

hipError_t geoball_sf(int n, const double* q0, double theta, double gamma, float* out, hipStream_t s) {
    const double qn = std::sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
    // radial distribution function on a uniform grid of [0, sin theta]
    std::vector<double> tab(2 * (size_t)GEOBALL_TABLE);
    double* tr = tab.data();
    double* tF = tab.data() + GEOBALL_TABLE;
    const double rmax = std::sin(theta), ct = std::cos(theta);
    auto density = [&](double r) {
        const double c = ct / std::sqrt(1.0 - r * r);
        return r * 2.0 * std::acos(c < 1.0 ? c : 1.0);
    };
    double prev = 0.0, acc = 0.0;
    for (int j = 0; j < GEOBALL_TABLE; ++j) {
        tr[j] = rmax * (double)j / (double)(GEOBALL_TABLE - 1);
        const double d = density(tr[j]);
        if (j > 0) acc += 0.5 * (d + prev) * (tr[j] - tr[j - 1]);
        tF[j] = acc;
        prev = d;
    }
    for (int j = 0; j < GEOBALL_TABLE; ++j) tF[j] /= acc;
    void* dtab = nullptr;
    hipError_t e = regdock_rt::dev_alloc(&dtab, tab.size() * sizeof(double));
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        const double* d = static_cast<const double*>(dtab);
        k_geoball_sf<<<(n + 255) / 256, 256, 0, s>>>(n, q0[0] / qn, q0[1] / qn, q0[2] / qn, q0[3] / qn, ct,
                                                     gamma > 0.0 ? gamma : (double)n, 1.0 / std::sqrt(2.0),
                                                     1.0 / psi_constant(), d, d + GEOBALL_TABLE, GEOBALL_TABLE, out);
        e = hipGetLastError();
    }
    const hipError_t es = hipStreamSynchronize(s);
    regdock_rt::dev_release(dtab);
    return e != hipSuccess ? e : es;
}

}  // namespace regdock
