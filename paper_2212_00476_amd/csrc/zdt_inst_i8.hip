// Kernel instances for 8-bit coded cost volumes (Sec. IV-C).
#define ZDT_ELEM zdt::i8c
#define ZDT_SUFFIX i8
#include "zdt_inst.hpp"
