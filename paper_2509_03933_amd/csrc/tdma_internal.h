// Internal declarations shared by the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/tdma.h"

namespace tdma {

// Where one launch's systems live.  System number k (0 <= k < nsys) maps to
// a system id (sys_list ? sys_list[k] : k).  Uniform layout: id = s0 + nsys0*s1
// starts at s0*sys_stride0 + s1*sys_stride1, rows row_stride apart.  Ragged:
// id starts at offsets[id] with offsets[id+1]-offsets[id] rows, row stride 1.
struct SysMap {
    int64_t n;              // rows per system (uniform); upper bound when ragged
    int64_t nsys;           // systems covered by this launch
    int64_t nsys0;
    int64_t row_stride, sys_stride0, sys_stride1;
    const int64_t *offsets; // device, ragged form only
    const int32_t *sys_list;// device, optional
    const unsigned long long *count;  // device, optional: systems actually listed (<= nsys)
};

struct Coef {
    int mode;               // TDMA_COEF_LIKE_D or TDMA_COEF_SHARED
    const void *a, *b, *c;
    const void *shift;      // per-system diagonal shift or null
};

// Tile shape of the fused kernel: S systems x P partitions x M rows per lane.
struct TileShape {
    int M = 8;
    int S_log2 = 4;
    int P = 4;
    bool contig = false;    // stage loads/stores through LDS (row_stride == 1)
    int kernel = 0;         // 0: generic fused kernel, 1: shared-operator kernel,
                            // 2: its streaming form (resident blocks walk the tiles),
                            // 3: shared operator + per-system shift, streaming with the
                            // next tile's rows loaded as Stage C frees registers, 4: the
                            // same loading each tile at its start (shifted.hip),
                            // 5: per-row coefficients, streaming (perrow.hip),
                            // 6: kernel 2 with one register set refilled as
                            // Stage C stores (partitions covering n exactly),
                            // 7: kernel 3 keeping only the right-hand sides and
                            // recomputing the pivots (FP64, P*M = n)
    bool pdd = false;       // kernel 0 only: Stage B by the PDD approximation
    int threads() const { return (1 << S_log2) * P; }
};

enum class Layout { Strided = 0, Contig = 1 };

// launchers (fused.hip)
hipError_t launch_fused(int dtype, const SysMap &map, const Coef &coef, const TileShape &shape,
                        const void *d, void *x, int *err_flag, hipStream_t stream);
bool fused_supported(int dtype, const TileShape &shape);
int fused_max_threads(int dtype, int M);
// LDS bytes of a fused launch; shared_rows: with the operator's rows in LDS.
size_t fused_lds_bytes(int dtype, const TileShape &shape, bool shared_rows = false);

// shared-operator launchers (shared.hip)
hipError_t launch_shared(int dtype, const SysMap &map, const Coef &coef, const TileShape &shape,
                         const void *d, void *x, int *err_flag, hipStream_t stream);
bool shared_supported(int dtype, const TileShape &shape);
// whether the rolling form (kernel 6) runs this map: strided rows of a plain
// uniform layout, P*M = n, 32-bit walk indices
bool shared_roll_ok(const SysMap &map, const TileShape &shape);
// lanes per block of the shared-operator kernels (kernel 2 with contiguous
// rows: the form that streams them, which holds two tiles in registers)
int shared_max_threads(int dtype, int M, int kernel, bool contig);
size_t shared_lds_bytes(int dtype, const TileShape &shape);
// the streaming solve's memory traffic alone (shared.hip), for measurement
bool copy_streamed_supported(const SysMap &map, const TileShape &shape);
hipError_t launch_copy_streamed(int dtype, const SysMap &map, const TileShape &shape,
                                const void *d, void *x, hipStream_t stream);

// shared operator with a per-system shift, strided layouts (shifted.hip)
bool shift_supported(int dtype, const TileShape &shape);
bool shift_layout_ok(const SysMap &map, const TileShape &shape);
size_t shift_lds_bytes(int dtype, const TileShape &shape);
hipError_t launch_shift(int dtype, const SysMap &map, const Coef &coef, const TileShape &shape,
                        const void *d, void *x, int *err_flag, hipStream_t stream);

// One tile of a ragged batch solved in a single launch (fused.hip): `count`
// systems (at most 2^S_log2) from entry `first` of the plan's system list,
// each of at most M << P_log2 rows; a block of 2^S_log2 << P_log2 lanes.
struct RaggedTile {
    int32_t first, count;
    int32_t P_log2, S_log2;
};
// per-row coefficients without a shift, contiguous rows; M = 16 (FP64) or
// 16, 32 (FP32); `threads` lanes per block for every tile of the list
bool fused_tiles_supported(int dtype, int M);
hipError_t launch_fused_tiles(int dtype, int M, const SysMap &map, const Coef &coef, const void *d,
                              void *x, const RaggedTile *tiles, int64_t ntiles, int threads,
                              size_t lds, int *err_flag, hipStream_t stream);

// per-row coefficients (a, b, c laid out like d), strided layouts, walking
// workgroups with 128-byte tile rows (perrow.hip)
bool perrow_supported(int dtype, const TileShape &shape);
bool perrow_layout_ok(const SysMap &map, const TileShape &shape);
size_t perrow_lds_bytes(const TileShape &shape);
hipError_t launch_perrow(int dtype, const SysMap &map, const Coef &coef, const TileShape &shape,
                         const void *d, void *x, int *err_flag, hipStream_t stream);

// several right-hand sides over one shared operator (multi.hip): S systems x
// P partitions (P <= 64) x M rows per lane, one tile per block
struct MultiShape {
    int M = 16;
    int P_log2 = 0;
    int S_log2 = 0;
};
// built-in shape for systems of n rows (false: n needs more than 64 partitions)
bool multi_shape(int dtype, int64_t n, int64_t nsys, MultiShape *out);
size_t multi_lds(int dtype, const MultiShape &shape, int nr);
// vec: two right-hand sides adjacent (rhs_stride 1) and pair-aligned
hipError_t launch_multi(int dtype, const SysMap &map, const Coef &coef, const MultiShape &shape,
                        int nrhs, int64_t rhs_stride, bool vec, const void *d, void *x,
                        int *err_flag, hipStream_t stream);

}  // namespace tdma
