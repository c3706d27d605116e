// Serving loop of libmcdose (continuous batching of dose requests).
#include "runtime.h"

void mcd_ctx::shutdown_serving() {}
