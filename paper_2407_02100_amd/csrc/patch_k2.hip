// Patch smoother launchers for degree 2.
#define VPS_PATCH_K 2
#include "patch_impl.h"
