// Patch smoother launchers for degree 4.
#define VPS_PATCH_K 4
#include "patch_impl.h"
