// aa_batch_p2.hip -- the batched / one-workgroup AA kernel of aa_batch.hip
// with two row pairs per lane per tile (namespace aa::p2); the schedule
// autotuner picks between it and the four-pair build.
#define AA_PAIRS 2
#define AA_BATCH_SECONDARY 1
#include "aa_batch.hip"
