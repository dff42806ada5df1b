// Kernel instances for zdt::bf16 cost volumes.
#define ZDT_ELEM zdt::bf16
#define ZDT_SUFFIX bf16
#include "zdt_inst.hpp"
