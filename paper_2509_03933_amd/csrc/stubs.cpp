// Entry points whose implementations are not built yet.
#include "api_internal.h"

using namespace tdma;



extern "C" {

int tdma_graph_create(const tdma_work_item *, int, int, tdma_graph **) {
    return fail(TDMA_EUNSUPPORTED, "tdma_graph_create is not built yet");
}

int tdma_graph_launch(tdma_graph *, void *) {
    return fail(TDMA_EUNSUPPORTED, "tdma_graph_launch is not built yet");
}

void tdma_graph_destroy(tdma_graph *) {}



}  // extern "C"
