// Error-evaluation kernels (covariance and projection error, Section 1.1).
#include "fdsk_device.hpp"
#include "fdsk_eval.hpp"
