// Serving loop (continuous batching) of the MRS filament library.
#include "mrs_runtime.h"
