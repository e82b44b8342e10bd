// Entry points whose implementations are not built yet.
#include "api_internal.h"

using namespace tdma;

namespace tdma {
bool lookup_tuned(int, const tdma_layout *, const tdma_coeffs *, int, TileShape *) { return false; }
void clear_tuned() {}
}  // namespace tdma

extern "C" {

int tdma_solve_partitioned(const tdma_layout *, const tdma_coeffs *, int, const void *, void *,
                           const tdma_part_opts *, void *) {
    return fail(TDMA_EUNSUPPORTED, "tdma_solve_partitioned is not built yet");
}

int tdma_solve_refined(const tdma_layout *, const tdma_coeffs *, const double *, double *,
                       const tdma_refine_opts *, tdma_refine_report *, void *) {
    return fail(TDMA_EUNSUPPORTED, "tdma_solve_refined is not built yet");
}

int tdma_graph_create(const tdma_work_item *, int, int, tdma_graph **) {
    return fail(TDMA_EUNSUPPORTED, "tdma_graph_create is not built yet");
}

int tdma_graph_launch(tdma_graph *, void *) {
    return fail(TDMA_EUNSUPPORTED, "tdma_graph_launch is not built yet");
}

void tdma_graph_destroy(tdma_graph *) {}

int tdma_autotune(const tdma_layout *, const tdma_coeffs *, int, const void *, void *, int, void *) {
    return fail(TDMA_EUNSUPPORTED, "tdma_autotune is not built yet");
}

}  // extern "C"
