// The register stages for codes of length 2^9, built in a unit of their own
// (the kernels and launchers are those of rq.hip).
#define POLAR_RQ_NL 9
#include "rq.hip"
