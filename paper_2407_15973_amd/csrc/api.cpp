// Library-level C ABI entry points of libmpbjac.
#include "../../include/mpbjac.h"

extern "C" int bjac_abi_version(void) { return MPBJAC_ABI_VERSION; }

extern "C" const char *bjac_strerror(int code) {
  switch (code) {
    case BJAC_OK: return "ok";
    case BJAC_NOT_CONVERGED: return "not converged: maxit reached";
    case BJAC_EINVAL: return "invalid argument";
    case BJAC_ENOTSPD: return "a diagonal block is not positive definite (non-positive pivot)";
    case BJAC_EBREAKDOWN: return "PCG breakdown: p'Ap <= 0, (r,z) <= 0 or non-finite";
    case BJAC_EHIP: return "HIP runtime error";
    case BJAC_ENOMEM: return "workspace too small";
    default: return "unknown error code";
  }
}
