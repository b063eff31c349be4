// pino_interp.h implementation.  Included once, by pino_collapse.hip.
#pragma once

#include <mutex>
#include <string>

#include "../../include/pino_interp.h"
#include "kernels_interp.h"

// Device scratch of pino_table_interp_noalloc: the shared elimination
// coefficients of the d-knots (4 kNoAllocMaxNd doubles), then the
// interleaved (F, M) table (2 kNoAllocMaxCells doubles).  Every GPU the
// library runs on holds its own copy until the process ends.  In host code
// the name is only a stand-in: kernels get the device address that
// hipGetSymbolAddress returns for the current device.
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 20;
constexpr int kNoAllocMaxNd = 4096;
constexpr int64_t kNoAllocDoubles = 4 * (int64_t)kNoAllocMaxNd + 2 * kNoAllocMaxCells;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

thread_local std::string g_interp_error = "no error";

pino_status interp_arg(const std::string& why)
{
    g_interp_error = why;
    return PINO_ERR_ARG;
}

pino_status interp_hip(hipError_t e, const char* what)
{
    g_interp_error = std::string(what) + ": " + hipGetErrorString(e);
    return PINO_ERR_HIP;
}

#define INTERP_HIP(call)                        \
    do {                                        \
        hipError_t e_ = (call);                 \
        if (e_ != hipSuccess)                   \
            return interp_hip(e_, #call);       \
    } while (0)

// enough workgroups to fill the device, no more than the queries need
// bins per knot interval of the spline's per-block interval index: random
// knots (the Sec. 4.3 benchmark) cluster, and at 8 bins per interval more
// than three knots rarely follow inside one bin
constexpr int kInterpBins = 8;

pino_status interp_grid(int32_t device, int64_t m, unsigned& grid)
{
    int cus = 0;
    INTERP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    const int64_t need = (m + 255) / 256;
    grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cus * 8));
    return PINO_OK;
}

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
constexpr int kNoAllocMaxDevices = 64;

pino_status scratch_on(int32_t device, double** out)
{
    static std::mutex mu;
    static double* ptr[kNoAllocMaxDevices] = {};
    if (device >= kNoAllocMaxDevices)
        return interp_arg("device ordinal beyond the 64 the static scratch table tracks");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        double* p = nullptr;
        INTERP_HIP(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
        ptr[device] = p;
    }
    *out = ptr[device];
    return PINO_OK;
}

}  // namespace

extern "C" {

pino_status pino_spline_build(int32_t device, const double* x, const double* y, int32_t n, double* M, double* work,
                              void* hip_stream)
{
    if (device < 0 || !x || !y || !M || !work || n < 2 || n > 2048)
        return interp_arg("need device >= 0, non-NULL x, y, M, work and 2 <= n <= 2048");
    INTERP_HIP(hipSetDevice(device));
    hipLaunchKernelGGL(pino::k_spline_build, dim3(1), dim3(64), 0, static_cast<hipStream_t>(hip_stream), x, n, y,
                       (int64_t)n, 1, M, (int64_t)n, 1, work, 1);
    INTERP_HIP(hipGetLastError());
    return PINO_OK;
}

pino_status pino_spline_eval(int32_t device, const double* x, const double* y, const double* M, int32_t n,
                             const double* q, double* out, int64_t m, void* hip_stream)
{
    if (device < 0 || !x || !y || !M || n < 2 || n > 2048 || m < 0 || (m > 0 && (!q || !out)))
        return interp_arg("need device >= 0, non-NULL knots (2 <= n <= 2048), m >= 0 and q, out for m > 0");
    if (m == 0)
        return PINO_OK;
    INTERP_HIP(hipSetDevice(device));
    unsigned grid = 0;
    const pino_status st = interp_grid(device, m, grid);
    if (st != PINO_OK)
        return st;
    // an interval index when each thread has at least 32 queries to amortise
    // the block's build and its bins fit beside the knots in 64 KiB of LDS
    const int64_t bins_fit = (65536 - 24 * (int64_t)n) / (int64_t)sizeof(int);
    const int nb = m >= (int64_t)grid * 256 * 32 ? (int)std::min<int64_t>(kInterpBins * (int64_t)(n - 1), bins_fit) : 0;
    hipLaunchKernelGGL(pino::k_spline_eval, dim3(grid), dim3(256),
                       (size_t)3 * n * sizeof(double) + (size_t)std::max(nb, 0) * sizeof(int),
                       static_cast<hipStream_t>(hip_stream), x, y, M, n, std::max(nb, 0), q, out, m);
    INTERP_HIP(hipGetLastError());
    return PINO_OK;
}

pino_status pino_table_build(int32_t device, int32_t nx, int32_t ny, int32_t nd, const double* dk, const double* F,
                             double* tab, double* work, void* hip_stream)
{
    if (device < 0 || !dk || !F || !tab || !work || nx < 2 || ny < 2 || nx > 1024 || ny > 1024 || nd < 2 ||
        nd > 4096)
        return interp_arg("need device >= 0, non-NULL arrays, 2 <= nx, ny <= 1024 and 2 <= nd <= 4096");
    INTERP_HIP(hipSetDevice(device));
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int rows = nx * ny;
    // the shared elimination coefficients (4 nd doubles) go to work
    hipLaunchKernelGGL(pino::k_spline_coef, dim3(1), dim3(64), 0, st, dk, nd, 1.0, work);
    INTERP_HIP(hipGetLastError());
    pino::launch_table_splines(work, 1.0, nd, F, tab, rows, st);
    INTERP_HIP(hipGetLastError());
    return PINO_OK;
}

pino_status pino_table_eval(int32_t device, const double* xk, int32_t nx, const double* yk, int32_t ny,
                            const double* dk, int32_t nd, const double* tab, const double* qx, const double* qy,
                            const double* qd, double* out, int64_t m, void* hip_stream)
{
    if (device < 0 || !xk || !yk || !dk || !tab || nx < 2 || ny < 2 || nx > 1024 || ny > 1024 || nd < 2 ||
        nd > 4096 || m < 0 || (m > 0 && (!qx || !qy || !qd || !out)))
        return interp_arg("need device >= 0, non-NULL knots and table, 2 <= nx, ny <= 1024, 2 <= nd <= 4096, "
                          "m >= 0 and non-NULL queries and out for m > 0");
    if (m == 0)
        return PINO_OK;
    INTERP_HIP(hipSetDevice(device));
    unsigned grid = 0;
    const pino_status st = interp_grid(device, m, grid);
    if (st != PINO_OK)
        return st;
    pino::TabArgs t{};  // no interval index: binary search on the knots
    t.xk = xk;
    t.yk = yk;
    t.dk = dk;
    t.nx = nx;
    t.ny = ny;
    t.nd = nd;
    t.scale = 1.0;
    t.inv_scale = 1.0;
    t.tab = tab;
    t.indexed = 0;
    const size_t lds = pino::table_lds_bytes(t);
    hipLaunchKernelGGL(pino::k_table_eval, dim3(grid), dim3(256), lds,
                       static_cast<hipStream_t>(hip_stream), t, qx, qy, qd, out, m);
    INTERP_HIP(hipGetLastError());
    return PINO_OK;
}

pino_status pino_table_interp_noalloc(int32_t device, const double* xk, int32_t nx, const double* yk, int32_t ny,
                                      const double* dk, int32_t nd, const double* F, const double* qx,
                                      const double* qy, const double* qd, double* out, int64_t m, void* hip_stream)
{
    if (device < 0 || !xk || !yk || !dk || !F || nx < 2 || ny < 2 || nx > 1024 || ny > 1024 || nd < 2 ||
        nd > kNoAllocMaxNd || m < 0 || (m > 0 && (!qx || !qy || !qd || !out)))
        return interp_arg("need device >= 0, non-NULL knots and values, 2 <= nx, ny <= 1024, 2 <= nd <= 4096, "
                          "m >= 0 and non-NULL queries and out for m > 0");
    const int64_t cells = (int64_t)nx * ny * nd;
    if (cells > kNoAllocMaxCells)
        return interp_arg("table of " + std::to_string(cells) + " values exceeds the " +
                          std::to_string(kNoAllocMaxCells) + " the static scratch holds");
    if (m == 0)
        return PINO_OK;
    INTERP_HIP(hipSetDevice(device));
    double* base = nullptr;
    pino_status ps = scratch_on(device, &base);
    if (ps != PINO_OK)
        return ps;
    double* coef = base;
    double* tab = base + 4 * (int64_t)kNoAllocMaxNd;
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // the kernels of pino_table_build, with the scratch in place of work/tab
    hipLaunchKernelGGL(pino::k_spline_coef, dim3(1), dim3(64), 0, st, dk, nd, 1.0, coef);
    INTERP_HIP(hipGetLastError());
    pino::launch_table_splines(coef, 1.0, nd, F, tab, nx * ny, st);
    INTERP_HIP(hipGetLastError());
    // and those of pino_table_eval
    unsigned grid = 0;
    ps = interp_grid(device, m, grid);
    if (ps != PINO_OK)
        return ps;
    pino::TabArgs t{};
    t.xk = xk;
    t.yk = yk;
    t.dk = dk;
    t.nx = nx;
    t.ny = ny;
    t.nd = nd;
    t.scale = 1.0;
    t.inv_scale = 1.0;
    t.tab = tab;
    t.indexed = 0;
    hipLaunchKernelGGL(pino::k_table_eval, dim3(grid), dim3(256), pino::table_lds_bytes(t), st, t, qx, qy, qd, out,
                       m);
    INTERP_HIP(hipGetLastError());
    return PINO_OK;
}

const char* pino_interp_last_error(void)
{
    return g_interp_error.c_str();
}

}  // extern "C"
