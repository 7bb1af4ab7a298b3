// common.hpp -- shared host-side declarations of the sgmi library (errors,
// argument checks).  Device code lives in the .hip files.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <string>

#include "sgmi.h"

namespace sg {

int fail(int code, const char *fmt, ...);
void clear_error();

inline bool lattice_ok(int32_t L) { return L >= 4 && L <= SG_MAX_L && (L % 2) == 0; }

}  // namespace sg
