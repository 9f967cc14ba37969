// Internal helpers shared by the libsnake HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/snake.h"

namespace snake {

// ---- host-side error reporting ------------------------------------------
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();
unsigned int *device_error_word();   // device address of this device's error word

#define SNAKE_REQUIRE(cond, code, ...)                                           \
    do {                                                                         \
        if (!(cond)) {                                                           \
            ::snake::set_error(__VA_ARGS__);                                     \
            return (code);                                                       \
        }                                                                        \
    } while (0)

#define SNAKE_NOT_NULL(p) SNAKE_REQUIRE((p) != nullptr, SNAKE_ERR_NULL, "%s: %s is NULL", __func__, #p)

#define SNAKE_ALIGNED(p, a)                                                                  \
    SNAKE_REQUIRE((reinterpret_cast<uintptr_t>(p) % (a)) == 0, SNAKE_ERR_ALIGN,             \
                  "%s: %s is not %d-byte aligned", __func__, #p, (int)(a))

inline int launch_status(const char *fn)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: kernel launch failed: %s", fn, hipGetErrorString(e));
        return SNAKE_ERR_HIP;
    }
    clear_error();
    return SNAKE_OK;
}

// Number of compute units of the current device (cached per device).
int num_cus();

// LDS bytes one block may allocate (per_cu false) or one CU holds (true).
int lds_bytes(bool per_cu);

// Current value of a launch-shape tunable (snake_tunable).
int tune(int which);

// Blocks for a grid-stride loop: enough to fill every CU `per_cu` times, but
// no more than the work needs.
inline unsigned grid_for(int64_t work_items, int block, int per_cu)
{
    int64_t need = (work_items + block - 1) / block;
    int64_t cap = (int64_t)num_cus() * per_cu;
    if (need < 1) need = 1;
    return (unsigned)(need < cap ? need : cap);
}

// ---- device helpers -------------------------------------------------------
__device__ __forceinline__ int64_t effective_n(int64_t n, const int64_t *n_dev)
{
    if (n_dev) {
        int64_t d = *n_dev;
        return d < n ? (d < 0 ? 0 : d) : n;
    }
    return n;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

template <typename T>
__device__ __forceinline__ T wave_shfl_up(T v, int delta)
{
    return __shfl_up(v, delta, 64);
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ float wave_inclusive_sum(float v)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        float u = __shfl_up(v, d, 64);
        if (l >= d) v += u;
    }
    return v;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

}  // namespace snake
