// Batched engine: placeholder until the body-resident kernel lands.
#include "titan_sim.h"

namespace titan {

int build_batch_engine(titan_sim *s)
{
    s->batch = nullptr;
    return TITAN_OK;
}

int enqueue_batch_steps(titan_sim *s, int64_t, int64_t)
{
    return fail(TITAN_ESTATE, "batched engine not available");
}

void destroy_batch_engine(titan_sim *s) { s->batch = nullptr; }

}  // namespace titan
