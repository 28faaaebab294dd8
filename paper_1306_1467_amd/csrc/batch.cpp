// Batched jobs: placeholder until the batched kernels land.
#include "launch.h"

using namespace vjb;

struct boost_batch { int dummy; };

extern "C" {
size_t boost_batch_workspace_bytes(int32_t, const boost_job*, const boost_options*) { set_error("batched jobs not built yet"); return 0; }
int boost_batch_init(boost_batch**, int32_t, const boost_job*, const boost_options*, void*, size_t) { set_error("batched jobs not built yet"); return BOOST_E_INVALID; }
int boost_batch_round(boost_batch*, boost_stump*) { return BOOST_E_INVALID; }
int boost_batch_train(boost_batch*, int32_t, boost_stump*) { return BOOST_E_INVALID; }
int boost_batch_get_weights(boost_batch*, int32_t, double*) { return BOOST_E_INVALID; }
int boost_batch_get_timing(boost_batch*, double*) { return BOOST_E_INVALID; }
void boost_batch_destroy(boost_batch*) {}
}
