// Shared declarations of the batching form (persist.hip, graph.cpp).
#pragma once
#include "tdma_internal.h"

namespace tdma {

constexpr int kPersistThreads = 1024;
constexpr int kMaxWorkDescs = 64;

// One work item (or one length class of a ragged item) of the persistent launch.
struct WorkDesc {
    SysMap map;
    Coef coef;
    const void *d;
    void *x;
    int S_log2, P;
    int like_d, shift, contig;
    int after;         // index of the descriptor whose output this one reads, or -1
    int64_t ntiles;
};

// A run of consecutive queue positions that belong to one descriptor.
struct WorkSeg {
    int desc;
    int64_t tile_begin;    // first tile of the descriptor in this run
    int64_t count;
    int64_t global_begin;  // queue position of the run's first tile
};

struct WorkCounters {
    unsigned long long head;                    // next queue position
    unsigned long long done[kMaxWorkDescs];     // finished tiles per descriptor
};

int persist_rows_per_lane();
hipError_t persist_occupancy(int dtype, size_t lds, int *blocks_per_cu);
hipError_t launch_persist_reset(WorkCounters *ctr, int ndesc, hipStream_t st);
hipError_t launch_persist(int dtype, int grid, size_t lds, const WorkDesc *descs,
                          const WorkSeg *segs, int nsegs, int64_t total_tiles, WorkCounters *ctr,
                          int *err, hipStream_t st);

}  // namespace tdma
