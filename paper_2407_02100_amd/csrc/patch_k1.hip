// Patch smoother launchers for degree 1.
#define VPS_PATCH_K 1
#include "patch_impl.h"
