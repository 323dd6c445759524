// jit.cpp -- hipRTC compilation of generated kernels and the code-object cache.
//
// The paper builds one executable per matrix with the vendor compiler
// (Sec. VI-E).  Here the generated source is compiled in-process by hipRTC for
// gfx950, loaded with hipModuleLoadData, and cached by its source text so that
// repeated calls on the same matrix and options reuse the code object.
#include <amd_comgr/amd_comgr.h>
#include <elf.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "jit.h"

namespace permx {

namespace {

// ---- FP64 instructions of the main loop, from the machine code ----
struct Disasm {
    const std::vector<char> *elf = nullptr;
    uint64_t base = 0, off = 0, size = 0;  // .text: address, file offset, bytes
    std::string text;                      // the last instruction
    uint64_t target = 0;                   // its resolved branch target, if any
    bool has_target = false;
};

uint64_t dis_read(uint64_t from, char *to, uint64_t size, void *ud) {
    Disasm *d = static_cast<Disasm *>(ud);
    if (from < d->base || from >= d->base + d->size) return 0;
    const uint64_t n = std::min<uint64_t>(size, d->base + d->size - from);
    memcpy(to, d->elf->data() + d->off + (from - d->base), n);
    return n;
}
void dis_print(const char *ins, void *ud) { static_cast<Disasm *>(ud)->text = ins; }
void dis_addr(uint64_t a, void *ud) {
    Disasm *d = static_cast<Disasm *>(ud);
    d->target = a;
    d->has_target = true;
}

// The .text section of an ELF64 code object: address, file offset, size.
bool find_text(const std::vector<char> &e, uint64_t *addr, uint64_t *off, uint64_t *size) {
    if (e.size() < sizeof(Elf64_Ehdr) || memcmp(e.data(), ELFMAG, SELFMAG) != 0) return false;
    Elf64_Ehdr h;
    memcpy(&h, e.data(), sizeof h);
    if (h.e_shoff == 0 || h.e_shentsize != sizeof(Elf64_Shdr) || h.e_shstrndx >= h.e_shnum) return false;
    if (h.e_shoff + (uint64_t)h.e_shnum * sizeof(Elf64_Shdr) > e.size()) return false;
    auto sec = [&](int i) {
        Elf64_Shdr s;
        memcpy(&s, e.data() + h.e_shoff + (uint64_t)i * sizeof(Elf64_Shdr), sizeof s);
        return s;
    };
    const Elf64_Shdr strs = sec(h.e_shstrndx);
    for (int i = 0; i < h.e_shnum; ++i) {
        const Elf64_Shdr s = sec(i);
        if (strs.sh_offset + s.sh_name + 6 > e.size()) continue;
        if (strcmp(e.data() + strs.sh_offset + s.sh_name, ".text") != 0) continue;
        if (s.sh_offset + s.sh_size > e.size()) return false;
        *addr = s.sh_addr;
        *off = s.sh_offset;
        *size = s.sh_size;
        return true;
    }
    return false;
}

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
    count_loop_fp64(&co);
    co.compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    co.cache_hit = false;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        g_cache.emplace(src, co);
    }
    *out = co;
    return PERM_OK;
}

void count_loop_fp64(CodeObject *co) {
    co->loop_add = co->loop_mul = co->loop_fma = -1;
    co->all_add = co->all_mul = co->all_fma = -1;
    Disasm d;
    d.elf = &co->code;
    if (!find_text(co->code, &d.base, &d.off, &d.size)) return;
    amd_comgr_disassembly_info_t info;
    if (amd_comgr_create_disassembly_info("amdgcn-amd-amdhsa--gfx950", dis_read, dis_print, dis_addr, &info) !=
        AMD_COMGR_STATUS_SUCCESS)
        return;
    // kind of each instruction: 0 other, 1 add, 2 mul, 3 fma; backward branches
    struct Ins {
        uint64_t addr;
        int kind;
    };
    std::vector<Ins> ins;
    std::vector<std::pair<uint64_t, uint64_t>> loops;  // (target, branch address)
    // long branches (bodies beyond a branch's reach): s_getpc_b64 s[k:k+1]
    // (the next instruction's address), s_add_u32 sk, sk, offset, ...,
    // s_setpc_b64 s[k:k+1]
    std::string pc_reg;
    uint64_t pc_base = 0, pc_target = 0;
    bool pc_known = false;
    for (uint64_t a = d.base; a < d.base + d.size;) {
        uint64_t sz = 0;
        d.text.clear();
        d.has_target = false;
        if (amd_comgr_disassemble_instruction(info, a, &d, &sz) != AMD_COMGR_STATUS_SUCCESS || sz == 0) break;
        std::string t = d.text;
        const size_t b = t.find_first_not_of(" \t");
        t = b == std::string::npos ? "" : t.substr(b);
        const std::string op = t.substr(0, t.find_first_of(" \t"));
        int kind = 0;
        if (op.rfind("v_add_f64", 0) == 0) kind = 1;
        else if (op.rfind("v_mul_f64", 0) == 0) kind = 2;
        else if (op.rfind("v_fma_f64", 0) == 0 || op.rfind("v_fmac_f64", 0) == 0) kind = 3;
        ins.push_back({a, kind});
        if (d.has_target && d.target <= a && (op.rfind("s_cbranch", 0) == 0 || op == "s_branch"))
            loops.push_back({d.target, a});
        const std::string args = t.size() > op.size() ? t.substr(op.size()) : std::string();
        auto operands = [&]() {
            std::vector<std::string> v;
            std::string cur;
            for (char ch : args) {
                if (ch == ',') {
                    v.push_back(cur);
                    cur.clear();
                } else if (ch != ' ' && ch != '\t') {
                    cur += ch;
                }
            }
            if (!cur.empty()) v.push_back(cur);
            return v;
        };
        if (op == "s_getpc_b64") {
            const auto v = operands();
            pc_reg = v.empty() ? "" : v[0];  // s[k:k+1]
            pc_base = a + sz;
            pc_known = false;
        } else if (op == "s_add_u32" && !pc_reg.empty()) {
            const auto v = operands();
            const std::string lo = "s" + pc_reg.substr(2, pc_reg.find(':') - 2);
            if (v.size() == 3 && v[0] == lo && v[1] == lo) {
                char *end = nullptr;
                const unsigned long long off = strtoull(v[2].c_str(), &end, 0);
                if (end && *end == 0) {
                    pc_target = pc_base + (uint64_t)(int64_t)(int32_t)(uint32_t)off;
                    pc_known = true;
                }
            }
        } else if (op == "s_setpc_b64" && pc_known) {
            const auto v = operands();
            if (!v.empty() && v[0] == pc_reg && pc_target <= a) loops.push_back({pc_target, a});
            pc_known = false;
        }
        a += sz;
    }
    amd_comgr_destroy_disassembly_info(info);
    int tot[4] = {0, 0, 0, 0};
    for (const Ins &i : ins) tot[i.kind]++;
    co->all_add = tot[1];
    co->all_mul = tot[2];
    co->all_fma = tot[3];
    int best = -1;
    for (const auto &lp : loops) {
        int c[4] = {0, 0, 0, 0};
        for (const Ins &i : ins)
            if (i.addr >= lp.first && i.addr < lp.second) c[i.kind]++;
        bool inner = true;  // no other loop with FP64 work inside this one
        for (const auto &l2 : loops) {
            if (l2 == lp || l2.first < lp.first || l2.second > lp.second) continue;
            for (const Ins &i : ins)
                if (i.addr >= l2.first && i.addr < l2.second && i.kind) {
                    inner = false;
                    break;
                }
            if (!inner) break;
        }
        if (inner && c[1] + c[2] + c[3] > best) {
            best = c[1] + c[2] + c[3];
            co->loop_add = c[1];
            co->loop_mul = c[2];
            co->loop_fma = c[3];
        }
    }
}

}  // namespace permx
