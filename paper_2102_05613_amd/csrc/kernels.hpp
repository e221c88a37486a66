// kernels.hpp -- every device kernel of the SK MCMCMC hot path (gfx950), by stage.
#pragma once
#include "common.hpp"
#include "propose.hpp"
#include "score_split.hpp"
#include "score_f64.hpp"
#include "select.hpp"
#include "delta.hpp"
#include "biased.hpp"
#include "sets.hpp"
#include "couplings.hpp"
#include "recompute.hpp"
