// Launchers of the error-evaluation kernels (covariance and projection error).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
