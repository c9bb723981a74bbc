// Adjoint (vector-Jacobian product) of one Lenia step.
#include "lenia.h"
#include "lenia_internal.h"
#include "lenia_plan.h"

using namespace lenia;

extern "C" lenia_status lenia_backward(lenia_plan_t p, const float* A_t, const float* P_t,
                                       const void* saved, const float* gA_next,
                                       const float* gP_next, float* gA_t, float* gP_t,
                                       float* gbeta, void* stream)
{
    (void)p; (void)A_t; (void)P_t; (void)saved; (void)gA_next; (void)gP_next;
    (void)gA_t; (void)gP_t; (void)gbeta; (void)stream;
    return set_error(LENIA_ERR_UNSUPPORTED, "adjoint not built yet");
}
