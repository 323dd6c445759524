// jit.h -- hipRTC compilation of generated kernels (see jit.cpp).
#pragma once

#include <string>
#include <vector>

#include "perm.h"

namespace permx {

struct CodeObject {
    std::vector<char> code;  // gfx950 ELF code object
    int vgprs = -1, agprs = -1, sgprs = -1, scratch_bytes = -1, lds_bytes = -1, vgpr_spills = -1;
    double compile_ms = 0.0;
    bool cache_hit = false;
    // FP64 VALU instructions (v_add_f64, v_mul_f64, v_fma_f64 / v_fmac_f64)
    // of the kernel's innermost loop with the most of them, read from the
    // code object's own machine code; -1 when it has no such loop
    int loop_add = -1, loop_mul = -1, loop_fma = -1;
    // the same over the whole kernel (the loop's instructions counted once)
    int all_add = -1, all_mul = -1, all_fma = -1;
};

// Fills co->loop_* from co->code (the disassembler of the ROCm code-object
// manager, one instruction at a time over the .text section).
void count_loop_fp64(CodeObject *co);

// Compiles generated HIP source for gfx950 (no GPU needed); cached by source.
perm_status compile_source(const std::string &src, CodeObject *out, std::string *err);

}  // namespace permx
