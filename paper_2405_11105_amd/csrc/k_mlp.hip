// Learned eigencomponent weights (MLP forward/backward/Adam); filled in later.
#include "lcf_internal.h"
#include "lcf_kernels.h"
