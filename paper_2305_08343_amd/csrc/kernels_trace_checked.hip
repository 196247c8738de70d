// The traversal kernels of kernels_trace.hip compiled a second time with device checks: every
// inner-node reference, leaf triangle range, stack push and tested codebook index is compared
// with the limits of the launch record before it is used, and a failed check sets a bit of the
// context's check word instead of reading or writing out of range. The library runs these
// instances when the context's checks are switched on (sc_set_device_checks).
#define SC_DEVICE_CHECKS 1
#include "kernels_trace.hip"
