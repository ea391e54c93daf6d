// Internal runtime helpers shared by the C ABI translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mtf.h"
#include "skeleton.h"

namespace mtf {

extern thread_local std::string g_err;

struct HipError : std::runtime_error {
    explicit HipError(const std::string& s) : std::runtime_error(s) {}
};
struct StateError : std::runtime_error {
    explicit StateError(const std::string& s) : std::runtime_error(s) {}
};
struct OomError : std::runtime_error {
    explicit OomError(const std::string& s) : std::runtime_error(s) {}
};
struct NonFiniteError : std::runtime_error {
    explicit NonFiniteError(const std::string& s) : std::runtime_error(s) {}
};
struct UnsupportedError : std::runtime_error {
    explicit UnsupportedError(const std::string& s) : std::runtime_error(s) {}
};

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw ::mtf::HipError(std::string(#x) + ": " + hipGetErrorString(e_));         \
    } while (0)

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        if (count == n && p) return;
        reset();
        if (count == 0) return;
        hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            if (e == hipErrorOutOfMemory) throw OomError("device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
            throw HipError(std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        n = count;
    }
    void upload(const std::vector<T>& v, hipStream_t s) {
        alloc(v.size());
        if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        HIPCHK(hipGetDevice(&prev));
        if (prev != dev) HIPCHK(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

// Device, stream and unknown count of a problem (defined with the problem object).
void problem_info(mtf_problem p, int* device, hipStream_t* stream, int64_t* N);

inline int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

// Runs f and maps exceptions to status codes; no exception crosses the ABI.
template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const MeshError& e) {
        return fail(MTF_ERR_MESH, e.what());
    } catch (const ArgError& e) {
        return fail(MTF_ERR_ARG, e.what());
    } catch (const StateError& e) {
        return fail(MTF_ERR_STATE, e.what());
    } catch (const OomError& e) {
        return fail(MTF_ERR_OOM, e.what());
    } catch (const NonFiniteError& e) {
        return fail(MTF_ERR_NONFINITE, e.what());
    } catch (const UnsupportedError& e) {
        return fail(MTF_ERR_UNSUPPORTED, e.what());
    } catch (const HipError& e) {
        return fail(MTF_ERR_HIP, e.what());
    } catch (const std::bad_alloc&) {
        return fail(MTF_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(MTF_ERR_ARG, e.what());
    } catch (...) {
        return fail(MTF_ERR_ARG, "unknown error");
    }
}

}  // namespace mtf
