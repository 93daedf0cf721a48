// Substitution kernels for factors of block size 4 (the kernels and the
// launcher are in sweep.h).
#define HBMC_SWEEP_KERNELS
#include "sweep.h"

int hbmc::launch_bs4(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
                  const ApplyCg *cg, int K, int nr, bool fwd_only, const Flow *fl) {
    return launch_bs<4>(f, r, z, s, done, cg, K, nr, fwd_only, fl);
}
