// placeholder translation unit, filled below
#include "common.h"
