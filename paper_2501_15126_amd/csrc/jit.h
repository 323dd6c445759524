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
};

// Compiles generated HIP source for gfx950 (no GPU needed); cached by source.
perm_status compile_source(const std::string &src, CodeObject *out, std::string *err);

}  // namespace permx
