// Kernel instances for FP16 working volumes scaled per pixel by the DT gain.
#define ZDT_ELEM zdt::f16x
#define ZDT_SUFFIX f16x
#include "zdt_inst.hpp"
