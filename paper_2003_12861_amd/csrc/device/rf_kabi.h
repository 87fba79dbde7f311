// rf_kabi.h -- argument block of the generated likelihood kernels.  Shared by
// the host launcher and the generated device source (passed by value as the
// kernel argument buffer), so both sides agree on the layout.
#pragma once
#include <stdint.h>

#define RF_MAX_COLS 8
#define RF_MAX_PARAMS 64
#define RF_TGMAX 32  // ticket groups at most
#define RF_TICKET_WORDS (64 * (1 + RF_TGMAX))

struct RfArgs {
  const void* col[RF_MAX_COLS];  // observable columns (float or double)
  int64_t n;                     // number of events
  double* part;                  // block partials: [nsum + 1][nblk_max] (last: bad-event count)
  unsigned* ticket;              // RF_TICKET_WORDS counters, 0 between launches: [0] global
                                 // ticket, [64 (1 + g)] ticket of group g < RF_TGMAX
  double* out;                   // result: [nll, grad[P], n_bad, sums...]
  void* values;                  // per-event output of the values kernel
  const double* aux;             // auxiliary FP64 inputs (e.g. surrogate normalisation)
  const void* weights;           // MLP weights (bf16)
  double* hout;                  // optional copy of out in mapped host memory (or null),
                                 // written word by word with system-scope stores
  int32_t nblk_max;              // stride of part (>= gridDim.x)
  int32_t pad_;
  double theta[RF_MAX_PARAMS];   // parameter point
};
