// ms_lib.hip — single translation unit of libms: the device kernels and the host runtime.
#include "ms_step.hip"
#include "ms_rl.hip"
#include "ms_host.cpp"
#include "ms_server.cpp"
#include "ms_peak.hip"
