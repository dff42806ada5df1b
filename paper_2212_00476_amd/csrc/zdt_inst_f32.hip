// Kernel instances for float cost volumes.
#define ZDT_ELEM float
#define ZDT_SUFFIX f32
#include "zdt_inst.hpp"
