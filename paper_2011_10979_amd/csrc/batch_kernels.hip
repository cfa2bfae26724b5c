// Kernels of the batched (work-queue) solve.
#include "kernels.hpp"
