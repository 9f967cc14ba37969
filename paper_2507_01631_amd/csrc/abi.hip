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

}  // namespace snake

extern "C" {

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
