// The C interface declared in include/libdpc.h: argument checks, exact
// thresholds, workspace lifetime and the order of the steps.
#include "dpc_internal.hpp"

#include <cmath>
#include <limits>
#include <mutex>

namespace dpc {

// floor(r^2) or ceil(r^2) of the exact value of the double r, saturating at
// INT64_MAX.  For r >= 1 the product splits exactly into hi + lo with
// hi = fl(r*r) and lo = fma(r, r, -hi) (an error-free transformation), and
// the rounding of hi + lo to an integer is decided from the two parts.
dpc_status square_threshold(double r, bool round_up, int64_t *out) {
    constexpr int64_t kMax = std::numeric_limits<int64_t>::max();
    if (out == nullptr || std::isnan(r) || r < 0.0)
        return DPC_ERR_INVALID_ARG;
    if (std::isinf(r)) {
        *out = kMax;
        return DPC_OK;
    }
    if (r < 1.0) {  // 0 <= r^2 < 1
        *out = (round_up && r > 0.0) ? 1 : 0;
        return DPC_OK;
    }
    const double hi = r * r;
    const double lo = std::fma(r, r, -hi);
    const double two63 = 9223372036854775808.0;
    const double two53 = 9007199254740992.0;
    if (hi > two63) {
        *out = kMax;
        return DPC_OK;
    }
    if (hi == two63) {
        // r^2 = 2^63 + lo with |lo| <= 512
        const double f = round_up ? std::ceil(lo) : std::floor(lo);
        *out = f >= 0.0 ? kMax : kMax + (int64_t)(f + 1.0);
        return DPC_OK;
    }
    if (hi >= two53) {
        // hi is an integer below 2^63; lo is the exact remainder
        const double f = round_up ? std::ceil(lo) : std::floor(lo);
        *out = (int64_t)hi + (int64_t)f;
        return DPC_OK;
    }
    const double fh = std::floor(hi);
    if (fh != hi) {
        // hi is at least one ulp from an integer and |lo| is at most half an ulp
        *out = (int64_t)fh + (round_up ? 1 : 0);
    } else {
        int64_t v = (int64_t)hi;
        if (round_up && lo > 0.0)
            v += 1;
        if (!round_up && lo < 0.0)
            v -= 1;
        *out = v;
    }
    return DPC_OK;
}

hipMemPool_t workspace_pool() {
    static std::mutex mu;
    static hipMemPool_t pools[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (pools[dev] == nullptr) {
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p = nullptr;
        if (hipMemPoolCreate(&p, &props) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
        pools[dev] = p;
    }
    return pools[dev];
}

namespace {

bool bad_shape(int64_t n, int32_t d) {
    return n < 0 || n > (int64_t)std::numeric_limits<int32_t>::max() - 1 || d < 1 || d > kMaxDim;
}

dpc_status delta_threshold(double delta_min, int64_t *Td) {
    if (std::isnan(delta_min))
        return DPC_ERR_INVALID_ARG;
    if (delta_min <= 0.0) {
        *Td = 0;
        return DPC_OK;
    }
    return square_threshold(delta_min, true, Td);
}

}  // namespace
}  // namespace dpc

using namespace dpc;

extern "C" {

const char *dpc_status_str(int status) {
    switch (status) {
    case DPC_OK: return "ok";
    case DPC_ERR_INVALID_ARG: return "invalid argument";
    case DPC_ERR_RANGE: return "coordinate range too wide: squared distances could exceed int64";
    case DPC_ERR_NOT_FOREST: return "dependent edges do not form a forest of rising priority";
    case DPC_ERR_OOM: return "device workspace allocation failed";
    case DPC_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

int dpc_square_threshold(double r, int32_t round_up, int64_t *out) {
    return square_threshold(r, round_up != 0, out);
}

int dpc_density(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t *rho, hipStream_t stream) {
    if (bad_shape(n, d) || std::isnan(d_cut) || d_cut < 0.0)
        return DPC_ERR_INVALID_ARG;
    if (n > 0 && (points == nullptr || rho == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0)
        return DPC_OK;
    int64_t T;
    DPC_TRY(square_threshold(d_cut, false, &T));
    Workspace ws(stream);
    Index ix;
    DPC_TRY(build_index(points, n, d, T, ws, ix));
    int32_t *srho;
    DPC_TRY(ws.alloc(&srho, n));
    return launch_density(ix, T, srho, rho, stream);
}

int dpc_dependent(const int32_t *points, int64_t n, int32_t d, const int32_t *rho, int32_t rho_min, int32_t *dep,
                  int64_t *delta2, hipStream_t stream) {
    if (bad_shape(n, d) || rho_min < 0)
        return DPC_ERR_INVALID_ARG;
    if (n > 0 && (points == nullptr || rho == nullptr || dep == nullptr || delta2 == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0)
        return DPC_OK;
    Workspace ws(stream);
    Index ix;
    DPC_TRY(build_index(points, n, d, 0, ws, ix));
    DPC_TRY(build_priority(nullptr, rho, ws, ix));
    const int32_t skip_below = rho_min > 0 ? rho_min : std::numeric_limits<int32_t>::min();
    return launch_dependent(ix, nullptr, skip_below, dep, delta2, stream);
}

int dpc_cluster(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2, int32_t rho_min,
                double delta_min, int32_t *label, hipStream_t stream) {
    if (n < 0 || n > (int64_t)std::numeric_limits<int32_t>::max() - 1 || rho_min < 0)
        return DPC_ERR_INVALID_ARG;
    int64_t Td;
    if (delta_threshold(delta_min, &Td) != DPC_OK)
        return DPC_ERR_INVALID_ARG;
    if (n > 0 && (rho == nullptr || dep == nullptr || delta2 == nullptr || label == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0)
        return DPC_OK;
    Workspace ws(stream);
    return launch_cluster(n, rho, dep, delta2, rho_min, Td, true, label, ws);
}

int dpc_run(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
            uint32_t flags, int32_t *rho, int32_t *dep, int64_t *delta2, int32_t *label, hipStream_t stream) {
    if (bad_shape(n, d) || std::isnan(d_cut) || d_cut < 0.0 || rho_min < 0 || (flags & ~DPC_SKIP_NOISE_DEPENDENTS))
        return DPC_ERR_INVALID_ARG;
    int64_t T, Td;
    if (delta_threshold(delta_min, &Td) != DPC_OK)
        return DPC_ERR_INVALID_ARG;
    if (n > 0 && (points == nullptr || rho == nullptr || dep == nullptr || delta2 == nullptr || label == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0)
        return DPC_OK;
    DPC_TRY(square_threshold(d_cut, false, &T));
    Workspace ws(stream);
    Index ix;
    DPC_TRY(build_index(points, n, d, T, ws, ix));
    int32_t *srho;
    DPC_TRY(ws.alloc(&srho, n));
    DPC_TRY(launch_density(ix, T, srho, rho, stream));
    DPC_TRY(build_priority(srho, nullptr, ws, ix));
    const int32_t dep_rho_min = (flags & DPC_SKIP_NOISE_DEPENDENTS) ? rho_min : std::numeric_limits<int32_t>::min();
    DPC_TRY(launch_dependent(ix, srho, dep_rho_min, dep, delta2, stream));
    return launch_cluster(n, rho, dep, delta2, rho_min, Td, false, label, ws);
}

}  // extern "C"
