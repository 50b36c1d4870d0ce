// Autotuner (placeholder).
#include "tc_api_internal.h"
