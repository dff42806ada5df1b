// Kernel instances for T-scaled 16-bit integer cost volumes (Sec. IV-C).
#define ZDT_ELEM zdt::i16v
#define ZDT_SUFFIX i16
#include "zdt_inst.hpp"
