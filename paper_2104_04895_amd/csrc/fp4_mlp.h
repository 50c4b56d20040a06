// fp4_mlp.h -- internal include of the surrogate network implementation; the public
// declarations live in include/fp4.h.
#pragma once
#include "fp4.h"
