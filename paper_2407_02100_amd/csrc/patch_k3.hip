// Patch smoother launchers for degree 3.
#define VPS_PATCH_K 3
#include "patch_impl.h"
