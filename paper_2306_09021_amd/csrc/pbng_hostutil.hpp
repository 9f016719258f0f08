// Host-side helpers shared by the tetrahedral and the planar C ABI of
// libpbng: error reporting (no C++ exception crosses the interface) and an
// owning device allocation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
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

// One entry of a batched upload: n_words 32-bit words from byte offset
// src_off of the staged payload to dst.
struct CopyItem {
    void* dst;
    uint32_t src_off;
    uint32_t n_words;
};

// Device side of a batched upload (one launch for every entry).
hipError_t launch_scatter_words(const void* staged, int n_items, uint32_t max_words, hipStream_t s);

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
// writes a table of CopyItem entries and the packed arrays into one pinned
// staging buffer, copies it to the device in one transfer, places every
// array with one scatter launch and waits, so the staging buffers and every
// target are ready when it returns.  Replaces one synchronous pageable copy
// plus a free and an allocation per array.  Array sizes are whole 32-bit
// words.
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
    void flush(Pinned& stage, Dev& dstage, hipStream_t s)
    {
        std::vector<CopyItem> tab;
        uint32_t max_words = 0;
        const size_t table = (items.size() * sizeof(CopyItem) + 255) & ~size_t(255);
        if (table + payload.size() >= (size_t(1) << 32)) fail(PBNG_EUNSUPPORTED, "upload batch too large");
        for (const Item& it : items) {
            if (it.n % 4) fail(PBNG_EINVAL, "upload of %zu bytes is not whole 32-bit words", it.n);
            if (it.n == 0) continue;
            tab.push_back({it.d->p, uint32_t(table + it.off), uint32_t(it.n / 4)});
            max_words = std::max(max_words, uint32_t(it.n / 4));
        }
        if (!tab.empty()) {
            const size_t total = table + payload.size();
            stage.reserve(total);
            dstage.reserve(total);
            unsigned char* h = static_cast<unsigned char*>(stage.p);
            std::memcpy(h, tab.data(), tab.size() * sizeof(CopyItem));
            std::memcpy(h + table, payload.data(), payload.size());
            hipchk(hipMemcpyAsync(dstage.p, stage.p, total, hipMemcpyHostToDevice, s), "upload");
            hipchk(launch_scatter_words(dstage.p, int(tab.size()), max_words, s), "upload scatter");
            hipchk(hipStreamSynchronize(s), "upload");
        }
        payload.clear();
        items.clear();
    }
};

}  // namespace pbng
