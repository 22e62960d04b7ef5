// Serving runtime (continuous batching of CP-ALS jobs).
#include "alto_internal.h"
