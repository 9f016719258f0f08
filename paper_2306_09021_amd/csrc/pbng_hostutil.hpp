// Host-side helpers shared by the tetrahedral and the planar C ABI of
// libpbng: error reporting (no C++ exception crosses the interface) and an
// owning device allocation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
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
    size_t cap = 0;
    Dev() = default;
    Dev(const Dev&) = delete;
    Dev& operator=(const Dev&) = delete;
    ~Dev() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        cap = 0;
    }
    // fresh allocation of n bytes (the old one is freed)
    void alloc(size_t n)
    {
        release();
        if (n == 0) n = 16;
        hipchk(hipMalloc(&p, n), "hipMalloc");
        bytes = cap = n;
    }
    // at least n bytes, keeping the current allocation (and its address)
    // when it is large enough; the caller makes sure no queued work still
    // reads the old contents
    void reserve(size_t n)
    {
        if (n == 0) n = 16;
        if (p && n <= cap) {
            bytes = n;
            return;
        }
        alloc(n);
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

// Pinned host memory that grows on demand.
struct Pinned {
    void* p = nullptr;
    size_t cap = 0;
    Pinned() = default;
    Pinned(const Pinned&) = delete;
    Pinned& operator=(const Pinned&) = delete;
    ~Pinned()
    {
        if (p) (void)hipHostFree(p);
    }
    void reserve(size_t n)
    {
        if (p && n <= cap) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        hipchk(hipHostMalloc(&p, n, hipHostMallocDefault), "hipHostMalloc");
        cap = n;
    }
};

// Batched uploads: add() sizes the target (keeping its allocation when it
// is large enough, see Dev::reserve) and packs the host array; flush()
// copies the packed arrays into one pinned staging buffer, issues one
// asynchronous copy per target on the stream and waits for them, so the
// staging buffer and every target are ready when it returns.  Replaces one synchronous pageable copy plus a
// free and an allocation per array.
struct Uploader {
    struct Item {
        Dev* d;
        size_t off, n;
    };
    std::vector<unsigned char> payload;
    std::vector<Item> items;
    // d holds at least v's bytes from here on (its address may be used at
    // once); the contents follow at flush()
    template <class T>
    void add(Dev& d, const std::vector<T>& v)
    {
        const size_t n = v.size() * sizeof(T);
        d.reserve(n);
        const size_t off = (payload.size() + 255) & ~size_t(255);
        payload.resize(off + n);
        if (n) std::memcpy(payload.data() + off, v.data(), n);
        items.push_back({&d, off, n});
    }
    void flush(Pinned& stage, hipStream_t s)
    {
        if (items.empty()) return;
        stage.reserve(std::max<size_t>(payload.size(), 256));
        std::memcpy(stage.p, payload.data(), payload.size());
        for (const Item& it : items) {
            if (it.n)
                hipchk(hipMemcpyAsync(it.d->p, static_cast<unsigned char*>(stage.p) + it.off, it.n,
                                      hipMemcpyHostToDevice, s),
                       "upload");
        }
        hipchk(hipStreamSynchronize(s), "upload");
        payload.clear();
        items.clear();
    }
};

}  // namespace pbng
