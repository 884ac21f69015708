// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pip.h"

namespace pip {

// ---------------------------------------------------------------- errors
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define PIP_HIP_TRY(expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::pip::fail(PIP_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define PIP_TRY(expr)            \
    do {                         \
        int r_ = (expr);         \
        if (r_ != PIP_OK)        \
            return r_;           \
    } while (0)

// ---------------------------------------------------------------- device facts
struct DeviceInfo {
    int device = -1;
    int cu_count = 0;
    bool gfx950 = false;
    unsigned *validate_flags = nullptr;   // address of the __device__ flag word
};
// Info for the current device (cached per device); PIP_ENOTSUP if not gfx950.
int current_device(DeviceInfo **out);

// ---------------------------------------------------------------- problem description
struct Problem {
    const double *px, *py;
    int64_t n_points;
    const int64_t *offsets;
    int64_t n_polys;
    const double *vx, *vy;
    int64_t n_vertices;
    const int32_t *point_poly;
    uint8_t *inside;
};

int check_host_args(const Problem &p);
// Device-side validation (synchronises `stream`): PIP_ERANGE / PIP_EDOM.
int validate_on_device(const Problem &p, DeviceInfo *dev, hipStream_t stream);

// ---------------------------------------------------------------- kernel launchers (exact binary64)
int launch_per_pair(const Problem &p, hipStream_t stream);
int launch_segmented(const Problem &p, hipStream_t stream, int pairs_per_lane, int block);
int launch_staged(const Problem &p, hipStream_t stream, int pairs_per_lane, int lds_slots);
int launch_copy(void *dst, const void *src, int64_t nbytes, hipStream_t stream);
int launch_validate(const Problem &p, unsigned *flags, hipStream_t stream);

enum : unsigned { VALIDATE_ERANGE = 1u, VALIDATE_EDOM = 2u };

}  // namespace pip
