// Host build of the engine's FP64 integral arithmetic (csrc/shg_math.h) for
// CPU unit tests. Test-only: libshg.so never falls back to this code.
#pragma once
#include <stdint.h>
#include "../../paper_1701_06588_amd/csrc/shg_math.h"
#include "../../paper_1701_06588_amd/csrc/boys_table.h"

using namespace shg;

typedef void (*pair_fn)(const double *, const double *, int, const double *, const double *, int,
                        const double *, double, const double *, double *, double *);
const pair_fn *hm_table_op0();
const pair_fn *hm_table_op1();
const pair_fn *hm_table_op2();
const pair_fn *hm_table_op3();
const pair_fn *hm_table_op4();
