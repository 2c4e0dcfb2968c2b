// common.hpp -- host-side helpers shared by the library's translation units.
#pragma once

#include <stdint.h>

#include <string>

#include "aes_gfx950.hpp"

namespace ogm {

std::string& last_error();                                            // thread-local message
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int check_launch(const char* what);                                   // FSS_EDEVICE on a launch error
RoundKeys seed_key(uint64_t seed);   // AES-128 schedule of LE64(seed) || "OBLIVGM1"
int shuffle_release();               // the shuffle's own streams (shuffle.hip), for fss_shutdown

}  // namespace ogm
