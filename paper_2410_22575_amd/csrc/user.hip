// User functions: f written once over the hDual type of chessfad_device.h,
// compiled at run time (hipRTC, gfx950) and run by the library's H.v and
// Hessian entry points under a func_id of its own.
//
// The generated kernel uses the paper's L1 mapping (Sec. VI): one lane per
// (point, row i); the lane walks the row's chunks in order, calls f once per
// chunk on the CHUNK-INIT seeds (made on access from the point's
// coordinates, so f may read y[k] in any order), and keeps the row's H.v sum
// (chunk dot, then chunks in order) or stores H[p][i][cs .. cs + C).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <mutex>
#include <string>
#include <vector>

#include "chessfad.h"
#include "runtime.hpp"

namespace {

// chessfad_device.h, embedded at build time
const char* kDeviceHeader =
#include "device_header.inc"
    ;

const char* kPrologue = R"CHESSFADK(#include "chessfad_device.h"
namespace chessfad {
// CHUNK-INIT for one call, made on access: y[k] = <x_k, [k = i], [k = cs + l], 0>
template <int C>
struct seeds {
    const double* x;
    int i, cs;
    __device__ __forceinline__ hdual<C> operator[](int k) const {
        hdual<C> y(x[k]);
        y.d = k == i ? 1.0 : 0.0;
        for (int l = 0; l < C; ++l) y.g[l] = (k - cs == l) ? 1.0 : 0.0;
        return y;
    }
};
}  // namespace chessfad
using chessfad::hdual;
#line 1 "user function"
)CHESSFADK";

const char* kEpilogue = R"CHESSFADK(
namespace chessfad {
template <int C>
__device__ __forceinline__ void user_rows(const double* x, const double* v, double* out, long long npts, int n,
                                          int hess) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts * n) return;
    const long long p = q / n;
    const int i = (int)(q - p * n);
    const int nc = (n + C - 1) / C;
    const double* xp = x + p * n;
    double res = 0.0;
    for (int j = 0; j < nc; ++j) {
        const int cs = j * C;
        const seeds<C> y{xp, i, cs};
        const hdual<C> f = chessfad_user_f<hdual<C>>(y, n);
        if (hess) {
            double* row = out + (p * n + i) * n + cs;
            for (int l = 0; l < C; ++l)
                if (cs + l < n) row[l] = f.h[l];
        } else {
            double dot = 0.0;
            for (int l = 0; l < C; ++l)
                if (cs + l < n) dot += f.h[l] * v[p * n + cs + l];
            res += dot;
        }
    }
    if (!hess) out[q] = res;
}
}  // namespace chessfad
#define CHESSFAD_USER_KERNEL(C)                                                                        \
    extern "C" __global__ __launch_bounds__(256) void chessfad_user_##C(                               \
        const double* x, const double* v, double* out, long long npts, int n, int hess) {              \
        chessfad::user_rows<C>(x, v, out, npts, n, hess);                                               \
    }
CHESSFAD_USER_KERNEL(1)
CHESSFAD_USER_KERNEL(2)
CHESSFAD_USER_KERNEL(4)
CHESSFAD_USER_KERNEL(8)
CHESSFAD_USER_KERNEL(16)
)CHESSFADK";

constexpr int kUserChunks[] = {1, 2, 4, 8, 16};
constexpr int kMaxDevices = 16;

struct UserFn {
    bool used = false;
    std::vector<char> code;
    hipModule_t mod[kMaxDevices] = {};
    hipFunction_t fn[kMaxDevices][5] = {};
};

std::mutex g_user_mu;
UserFn g_user[CHESSFAD_MAX_USER];
thread_local std::string g_compile_log;

int chunk_slot(int C) {
    for (int k = 0; k < 5; ++k)
        if (kUserChunks[k] == C) return k;
    return -1;
}

}  // namespace

namespace chessfad {

bool user_registered(int func_id) {
    const int slot = func_id - CHESSFAD_USER_BASE;
    if (slot < 0 || slot >= CHESSFAD_MAX_USER) return false;
    std::lock_guard<std::mutex> lk(g_user_mu);
    return g_user[slot].used;
}

const char* user_compile_log() { return g_compile_log.c_str(); }

// Arguments are checked by the caller (run_single).
int run_user(int func_id, int n, int64_t npts, const double* x, const double* v, double* out, int chunk,
             hipStream_t stream, bool hess) {
    const int slot = func_id - CHESSFAD_USER_BASE;
    const int cslot = chunk_slot(chunk);
    if (cslot < 0) return CHESSFAD_E_CHUNK;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= kMaxDevices) return CHESSFAD_E_ARG;
    hipFunction_t fn = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_user_mu);
        UserFn& u = g_user[slot];
        if (!u.used) return CHESSFAD_E_FUNC;
        if (!u.mod[dev]) {
            e = hipModuleLoadData(&u.mod[dev], u.code.data());
            if (e != hipSuccess) {
                u.mod[dev] = nullptr;
                return hip_fail(e);
            }
        }
        if (!u.fn[dev][cslot]) {
            const std::string name = "chessfad_user_" + std::to_string(chunk);
            e = hipModuleGetFunction(&u.fn[dev][cslot], u.mod[dev], name.c_str());
            if (e != hipSuccess) return hip_fail(e);
        }
        fn = u.fn[dev][cslot];
    }
    const int64_t rows = npts * (int64_t)n;
    const int64_t grid = (rows + 255) / 256;
    if (grid > 0x7fffffffLL) return CHESSFAD_E_ARG;
    long long np = (long long)npts;
    int nn = n, hs = hess ? 1 : 0;
    void* args[] = {&x, &v, &out, &np, &nn, &hs};
    e = hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, 256, 1, 1, 0, stream, args, nullptr);
    return e == hipSuccess ? CHESSFAD_OK : hip_fail(e);
}

}  // namespace chessfad

using namespace chessfad;

extern "C" {

int chessfad_register_function(const char* source, int* func_id) {
    if (!source || !func_id) return CHESSFAD_E_NULL;
    const std::string text = std::string(kPrologue) + source + kEpilogue;
    hiprtcProgram prog = nullptr;
    const char* hdr[] = {kDeviceHeader};
    const char* hdr_name[] = {"chessfad_device.h"};
    if (hiprtcCreateProgram(&prog, text.c_str(), "chessfad_user.hip", 1, hdr, hdr_name) != HIPRTC_SUCCESS) {
        g_compile_log = "hiprtcCreateProgram failed";
        return CHESSFAD_E_COMPILE;
    }
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=fast",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    size_t log_size = 0;
    hiprtcGetProgramLogSize(prog, &log_size);
    std::string log(log_size, '\0');
    if (log_size) hiprtcGetProgramLog(prog, &log[0]);
    g_compile_log = log.c_str();
    if (rc != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        if (g_compile_log.empty()) g_compile_log = hiprtcGetErrorString(rc);
        return CHESSFAD_E_COMPILE;
    }
    size_t code_size = 0;
    hiprtcGetCodeSize(prog, &code_size);
    std::vector<char> code(code_size);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);

    std::lock_guard<std::mutex> lk(g_user_mu);
    for (int slot = 0; slot < CHESSFAD_MAX_USER; ++slot) {
        if (g_user[slot].used) continue;
        g_user[slot] = UserFn{};
        g_user[slot].used = true;
        g_user[slot].code = std::move(code);
        *func_id = CHESSFAD_USER_BASE + slot;
        return CHESSFAD_OK;
    }
    return CHESSFAD_E_ARG;
}

int chessfad_release_function(int func_id) {
    const int slot = func_id - CHESSFAD_USER_BASE;
    if (slot < 0 || slot >= CHESSFAD_MAX_USER) return CHESSFAD_E_FUNC;
    std::lock_guard<std::mutex> lk(g_user_mu);
    UserFn& u = g_user[slot];
    if (!u.used) return CHESSFAD_E_FUNC;
    for (int d = 0; d < kMaxDevices; ++d)
        if (u.mod[d]) (void)hipModuleUnload(u.mod[d]);
    u = UserFn{};
    return CHESSFAD_OK;
}

}  // extern "C"
