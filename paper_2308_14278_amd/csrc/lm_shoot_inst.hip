// lm_shoot_inst.hip -- the shooting kernels, the probes that repeat their
// arithmetic, and their launchers, for one (scheme, precision) pair: LM_S
// (LM_SCHEME_*) and LM_PR (LM_PREC_*, not LM_PREC_AUTO) come from the compiler
// command line.  The library compiles this file once per supported pair, so
// the heavy template instantiations build in parallel; lm_kernels.hip picks
// the pair at run time.
#include "lm_device.h"

#if !defined(LM_S) || !defined(LM_PR)
#error "compile with -DLM_S=<scheme> -DLM_PR=<precision>"
#endif

int LM_INST_CAT(lm_inst_shoot_map, LM_S, LM_PR)(const LmDesc& d, int nr, int terms, void* stream)
{
    MapLauncher f{d, (hipStream_t)stream};
    return dispatch_nr<LM_S, LM_PR>(nr, terms, f);
}

int LM_INST_CAT(lm_inst_shoot_batch, LM_S, LM_PR)(const LmDesc* descs, const int64_t* offs,
                                                  const int32_t* order, int nmaps,
                                                  unsigned long long* queue, int nr, int terms,
                                                  int layout, int grid, void* stream)
{
    BatchLauncher f{descs, offs, order, nmaps, queue, layout, grid, (hipStream_t)stream};
    return dispatch_nr<LM_S, LM_PR>(nr, terms, f);
}

int LM_INST_CAT(lm_inst_occupancy, LM_S, LM_PR)(int nr, int terms, int layout, int* wg_per_cu)
{
    Occupancy f{layout, wg_per_cu};
    return dispatch_nr<LM_S, LM_PR>(nr, terms, f);
}

// the probes do not depend on the rays per lane
int LM_INST_CAT(lm_inst_trace, LM_S, LM_PR)(const LmDesc& d, int terms, const int64_t* ii,
                                            const int64_t* jj, int64_t n, int32_t* p, int32_t* q,
                                            double* uv, void* stream)
{
    TraceLauncher f{d, ii, jj, n, p, q, uv, (hipStream_t)stream};
    return dispatch_p<LM_S, LM_PR, 4>(terms, f);
}

int LM_INST_CAT(lm_inst_deflect, LM_S, LM_PR)(const LmDesc& d, int terms, const double* th,
                                              int64_t n, double* alpha, void* stream)
{
    DeflectLauncher f{d, th, n, alpha, (hipStream_t)stream};
    return dispatch_p<LM_S, LM_PR, 4>(terms, f);
}
