// HIP kernels of the solver hot path.  Each iteration of a method is a short
// sequence of fused streaming passes; the scalars of the method live in a
// device State and are updated by the finishing reduction of each pass, so
// an iteration needs no host round trip.
#pragma once

#include "csr.hpp"
#include "kernels_basic.hpp"
#include "kernels_bicgstab.hpp"
#include "kernels_cg.hpp"
#include "kernels_cgnb.hpp"
#include "kernels_ir.hpp"
#include "kernels_persist.hpp"
#include "kernels_relax.hpp"
#include "kernels_util.hpp"
#include "sell.hpp"
#include "stencil.hpp"
#include "varcoef.hpp"
