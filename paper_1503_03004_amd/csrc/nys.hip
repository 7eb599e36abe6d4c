// FR-Nys (Alg. 3): shuffle, two FR-ADM sub-solves, Nystrom combine.
#include "engine.hpp"

namespace sfr {

sfr_status nys_setup(sfr_ctx* h)
{
    (void)h;
    return SFR_ERR_ARG;
}

}  // namespace sfr

extern "C" sfr_status sfr_solve_nys(sfr_handle h, const void* M, int64_t ldm, const int64_t* perm, void* U,
                                    double* B, void* V, void* S, int64_t lds, sfr_info* info, void* hip_stream)
{
    (void)M; (void)ldm; (void)perm; (void)U; (void)B; (void)V; (void)S; (void)lds; (void)info; (void)hip_stream;
    if (!h) return SFR_ERR_HANDLE;
    return SFR_ERR_HANDLE;
}
