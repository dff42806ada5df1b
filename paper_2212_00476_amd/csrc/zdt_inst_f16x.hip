// Kernel instances for FP16 working volumes with per-chunk exponents.
#define ZDT_ELEM zdt::f16x
#define ZDT_SUFFIX f16x
#include "zdt_inst.hpp"
