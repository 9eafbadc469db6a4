// Patch smoother launchers for degree 5.
#define VPS_PATCH_K 5
#include "patch_impl.h"
