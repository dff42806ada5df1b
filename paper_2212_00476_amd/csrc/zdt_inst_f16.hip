// Kernel instances for _Float16 cost volumes.
#define ZDT_ELEM _Float16
#define ZDT_SUFFIX f16
#include "zdt_inst.hpp"
