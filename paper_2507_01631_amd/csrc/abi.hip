// Library shell: version, thread-local error message, device error word.
#include <stdarg.h>
#include <string.h>

#include <mutex>

#include "common.h"

namespace snake {

static thread_local char g_msg[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
}

void clear_error() { g_msg[0] = '\0'; }

// One error word per device; kernels receive its address as an argument.
__device__ unsigned int g_device_error;

static constexpr int kMaxDevices = 64;
static unsigned int *g_err_ptr[kMaxDevices];
static int g_cus[kMaxDevices];
static int g_lds[kMaxDevices][2];
static std::mutex g_mu;

unsigned int *device_error_word()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_err_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_device_error)) != hipSuccess) return nullptr;
        g_err_ptr[dev] = static_cast<unsigned int *>(p);
    }
    return g_err_ptr[dev];
}

int num_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        g_cus[dev] = v;
    }
    return g_cus[dev];
}

int lds_bytes(bool per_cu)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 65536;
    std::lock_guard<std::mutex> lk(g_mu);
    int &c = g_lds[dev][per_cu ? 1 : 0];
    if (!c) {
        int v = 0;
        const hipDeviceAttribute_t a =
            per_cu ? hipDeviceAttributeMaxSharedMemoryPerMultiprocessor : hipDeviceAttributeMaxSharedMemoryPerBlock;
        if (hipDeviceGetAttribute(&v, a, dev) != hipSuccess || v <= 0) v = 65536;
        c = v;
    }
    return c;
}

// Launch-shape tunables (the only process-wide setting).
static const int32_t kTuneDefault[SNAKE_TUNE_COUNT] = {16, 8, 0, 8, 2048, 0, 16, 0, 1};
static const int32_t kTuneMin[SNAKE_TUNE_COUNT] = {1, 1, 0, 1, 64, 0, 1, 0, 0};
static const int32_t kTuneMax[SNAKE_TUNE_COUNT] = {64, 16, 2, 64, 2048, 32, 64, 64, 1};
static int32_t g_tune[SNAKE_TUNE_COUNT] = {16, 8, 0, 8, 2048, 0, 16, 0, 1};

int tune(int which) { return g_tune[which]; }

}  // namespace snake

extern "C" {

int snake_tune_set(int32_t which, int32_t value)
{
    SNAKE_REQUIRE(which >= 0 && which < SNAKE_TUNE_COUNT, SNAKE_ERR_INVALID_ARG, "snake_tune_set: unknown id %d",
                  which);
    if (value == 0 && snake::kTuneMin[which] > 0) value = snake::kTuneDefault[which];
    SNAKE_REQUIRE(value >= snake::kTuneMin[which] && value <= snake::kTuneMax[which], SNAKE_ERR_INVALID_ARG,
                  "snake_tune_set: value %d of tunable %d not in [%d, %d]", value, which, snake::kTuneMin[which],
                  snake::kTuneMax[which]);
    snake::g_tune[which] = value;
    snake::clear_error();
    return SNAKE_OK;
}

int32_t snake_tune_get(int32_t which)
{
    if (which < 0 || which >= SNAKE_TUNE_COUNT) return -1;
    return snake::g_tune[which];
}

int snake_stream_create_dedicated(snake_stream_t *stream)
{
    SNAKE_REQUIRE(stream != nullptr, SNAKE_ERR_NULL, "snake_stream_create_dedicated: stream is NULL");
    const int ncu = snake::num_cus();
    uint32_t mask[64];
    const uint32_t words = (uint32_t)((ncu + 31) / 32);
    SNAKE_REQUIRE(words >= 1 && words <= 64, SNAKE_ERR_INVALID_ARG, "snake_stream_create_dedicated: %d compute units",
                  ncu);
    for (uint32_t i = 0; i < words; ++i) mask[i] = 0xffffffffu;
    hipStream_t st = nullptr;
    const hipError_t e = hipExtStreamCreateWithCUMask(&st, words, mask);
    SNAKE_REQUIRE(e == hipSuccess, SNAKE_ERR_HIP, "snake_stream_create_dedicated: %s", hipGetErrorString(e));
    *stream = reinterpret_cast<snake_stream_t>(st);
    snake::clear_error();
    return SNAKE_OK;
}

int snake_stream_destroy(snake_stream_t stream)
{
    SNAKE_REQUIRE(stream != nullptr, SNAKE_ERR_NULL, "snake_stream_destroy: stream is NULL");
    const hipError_t e = hipStreamDestroy(reinterpret_cast<hipStream_t>(stream));
    SNAKE_REQUIRE(e == hipSuccess, SNAKE_ERR_HIP, "snake_stream_destroy: %s", hipGetErrorString(e));
    snake::clear_error();
    return SNAKE_OK;
}

int snake_abi_version(void) { return SNAKE_ABI_VERSION; }

const char *snake_last_error(void) { return snake::g_msg; }

int snake_check_device_error(snake_stream_t stream, uint32_t *bits)
{
    unsigned int *w = snake::device_error_word();
    SNAKE_REQUIRE(w != nullptr, SNAKE_ERR_HIP, "snake_check_device_error: no device error word");
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    SNAKE_REQUIRE(e == hipSuccess, SNAKE_ERR_HIP, "snake_check_device_error: %s", hipGetErrorString(e));
    unsigned int v = 0;
    e = hipMemcpy(&v, w, sizeof(v), hipMemcpyDeviceToHost);
    SNAKE_REQUIRE(e == hipSuccess, SNAKE_ERR_HIP, "snake_check_device_error: %s", hipGetErrorString(e));
    if (bits) *bits = v;
    if (v) {
        unsigned int zero = 0;
        e = hipMemcpy(w, &zero, sizeof(zero), hipMemcpyHostToDevice);
        SNAKE_REQUIRE(e == hipSuccess, SNAKE_ERR_HIP, "snake_check_device_error: %s", hipGetErrorString(e));
        snake::set_error("device error bits 0x%x", v);
        return SNAKE_ERR_DEVICE;
    }
    snake::clear_error();
    return SNAKE_OK;
}

}  // extern "C"
