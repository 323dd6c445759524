// jit.cpp -- hipRTC compilation of generated kernels and the code-object cache.
//
// The paper builds one executable per matrix with the vendor compiler
// (Sec. VI-E).  Here the generated source is compiled in-process by hipRTC for
// gfx950, loaded with hipModuleLoadData, and cached by its source text so that
// repeated calls on the same matrix and options reuse the code object.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <chrono>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "jit.h"

namespace permx {

namespace {

const char *const kRtcOptions[] = {
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
    // no packed FP32 instructions anywhere (only FP64 arithmetic is used)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
};

// Reads an unsigned msgpack integer that follows `key` in the code object's
// metadata note; -1 when absent.
long msgpack_uint_after(const std::vector<char> &co, const char *key) {
    const size_t kl = strlen(key);
    for (size_t i = 0; i + kl + 1 < co.size(); ++i) {
        // fixstr header (0xa0 | len) followed by the key bytes
        if ((unsigned char)co[i] != (0xa0u | (unsigned)kl)) continue;
        if (memcmp(&co[i + 1], key, kl) != 0) continue;
        size_t v = i + 1 + kl;
        const unsigned char b = (unsigned char)co[v];
        if (b < 0x80) return b;
        if (b == 0xcc && v + 1 < co.size()) return (unsigned char)co[v + 1];
        if (b == 0xcd && v + 2 < co.size())
            return ((unsigned char)co[v + 1] << 8) | (unsigned char)co[v + 2];
        if (b == 0xce && v + 4 < co.size())
            return ((long)(unsigned char)co[v + 1] << 24) | ((unsigned char)co[v + 2] << 16) |
                   ((unsigned char)co[v + 3] << 8) | (unsigned char)co[v + 4];
        return -1;
    }
    return -1;
}

std::mutex g_cache_mu;
std::unordered_map<std::string, CodeObject> g_cache;  // source text -> code object

}  // namespace

perm_status compile_source(const std::string &src, CodeObject *out, std::string *err) {
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_cache.find(src);
        if (it != g_cache.end()) {
            *out = it->second;
            out->cache_hit = true;
            out->compile_ms = 0.0;
            return PERM_OK;
        }
    }
    auto t0 = std::chrono::steady_clock::now();
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "perm_gray.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        *err = "hiprtcCreateProgram failed";
        return PERM_ECOMPILE;
    }
    const int nopt = (int)(sizeof(kRtcOptions) / sizeof(kRtcOptions[0]));
    hiprtcResult rc = hiprtcCompileProgram(prog, nopt, kRtcOptions);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        *err = std::string("hipRTC compile failed: ") + hiprtcGetErrorString(rc) + "\n" + log.substr(0, 4000);
        return PERM_ECOMPILE;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    CodeObject co;
    co.code.resize(cs);
    hiprtcGetCode(prog, co.code.data());
    hiprtcDestroyProgram(&prog);
    co.vgprs = (int)msgpack_uint_after(co.code, ".vgpr_count");
    co.agprs = (int)msgpack_uint_after(co.code, ".agpr_count");
    co.sgprs = (int)msgpack_uint_after(co.code, ".sgpr_count");
    co.scratch_bytes = (int)msgpack_uint_after(co.code, ".private_segment_fixed_size");
    co.lds_bytes = (int)msgpack_uint_after(co.code, ".group_segment_fixed_size");
    co.vgpr_spills = (int)msgpack_uint_after(co.code, ".vgpr_spill_count");
    co.compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    co.cache_hit = false;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        g_cache.emplace(src, co);
    }
    *out = co;
    return PERM_OK;
}

}  // namespace permx
