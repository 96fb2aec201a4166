// Split-Euler-Maruyama step kernels (filled in below).
#include "common.h"
namespace rb {}
