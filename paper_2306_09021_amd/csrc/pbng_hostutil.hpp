// Host-side helpers shared by the tetrahedral and the planar C ABI of
// libpbng: error reporting (no C++ exception crosses the interface) and an
// owning device allocation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "pbng.h"

namespace pbng {

// Thread-local text of the last error (pbng_last_error).
inline thread_local std::string g_err;

struct Error {
    int code;
    std::string msg;
};

[[noreturn]] inline void fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{code, buf};
}

inline void hipchk(hipError_t e, const char* what)
{
    if (e == hipSuccess) return;
    const int code = (e == hipErrorOutOfMemory) ? PBNG_ENOMEM : PBNG_EHIP;
    fail(code, "%s: %s", what, hipGetErrorString(e));
}

template <class F>
int32_t guard(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_err = "out of host memory";
        return PBNG_ENOMEM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return PBNG_EINVAL;
    } catch (...) {
        g_err = "unknown error";
        return PBNG_EINVAL;
    }
}

// Owning device allocation.
struct Dev {
    void* p = nullptr;
    size_t bytes = 0;
    Dev() = default;
    Dev(const Dev&) = delete;
    Dev& operator=(const Dev&) = delete;
    ~Dev() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t n)
    {
        release();
        if (n == 0) n = 16;
        hipchk(hipMalloc(&p, n), "hipMalloc");
        bytes = n;
    }
    template <class T>
    void upload(const std::vector<T>& v)
    {
        alloc(v.size() * sizeof(T));
        if (!v.empty()) hipchk(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
    }
    template <class T>
    T* as() const
    {
        return static_cast<T*>(p);
    }
};

}  // namespace pbng
