// Loop-kind dispatch, default launch configurations and their validation.
#include "jacc.h"
#include "kernels.h"

namespace jk {

static int64_t inner_extent(const Launch &L) {
    // length of the contiguous (innermost) dimension of the first argument
    int nd = 1;
    for (int i = 1; i < 4; ++i)
        if (L.ext[i] > 0) nd = i + 1;
    return L.ext[nd - 1];
}

Cfg default_config(int kind, const Launch &L, Cfg c) {
    const bool even = (inner_extent(L) % 2) == 0;
    switch (kind) {
        case JACC_LOOP_JACOBI2D:
            if (!c.bx) c.bx = 256;
            if (!c.by) c.by = 1;
            // measured: 4-row tiles for eager launches and for task-kernel
            // tiles at every partition count (8190-column grids and 512^2,
            // K = 1..8)
            if (!c.tile) c.tile = 4;
            if (!c.vec) c.vec = even ? 2 : 1;
            if (!c.order) c.order = 1;
            if (!c.march) c.march = 2;
            if (!c.rows) c.rows = 1;
            break;
        case JACC_LOOP_HEAT3D:
            if (!c.rows) {  // multi-row waves need workgroups of at most 256 threads
                const int bx = c.bx ? c.bx : 128, by = c.by ? c.by : 2;
                c.rows = (c.persistent || bx * by > 256) ? 1 : 4;
            }
            if (!c.bx) c.bx = c.rows > 1 ? 128 : 256;
            if (!c.by) c.by = c.rows > 1 ? 2 : 4;
            if (!c.tile) c.tile = c.rows > 1 ? 8 : 4;
            if (!c.vec) c.vec = even ? 2 : 1;
            if (!c.order) c.order = c.rows > 1 ? 3 : 1;  // y-blocked bricks: 8 % read overfetch instead of 41 %
            if (!c.march) c.march = 2;
            break;
        default:
            if (!c.bx) c.bx = kind == JACC_LOOP_GEMM ? 512 : 256;  // GEMM: 8 waves of 64x32 measured faster
            if (!c.by) c.by = 1;
            // measured: GEMM 16-deep slabs; SpMV 16 lanes per row (one gather
            // per lane for ~16 non-zeros) with non-temporal col/val loads
            if (!c.tile) c.tile = kind == JACC_LOOP_GEMM ? 16 : kind == JACC_LOOP_SPMV_CSR ? 16 : 1;
            if (!c.vec) c.vec = 1;
            if (!c.order) c.order = kind == JACC_LOOP_SPMV_CSR ? 2 : 1;
            if (!c.march) c.march = 1;
            if (!c.rows) c.rows = 1;
            break;
    }
    return c;
}

int check_config(const Launch &L) {
    const Cfg &c = L.cfg;
    if (c.persistent != 0 && c.persistent != 1) return 1;
    if (c.persistent && L.kind != JACC_LOOP_JACOBI2D && L.kind != JACC_LOOP_HEAT3D) return 1;
    switch (L.kind) {
        case JACC_LOOP_JACOBI2D:
        case JACC_LOOP_HEAT3D:
            if (c.bx < 64 || c.bx % 64 || c.by < 1 || c.bx * c.by > 1024) return 1;
            if (c.tile < 1 || c.tile > 65536) return 1;
            if (c.vec != 1 && c.vec != 2) return 1;
            if (c.vec == 2 && inner_extent(L) % 2) return 1;
            if (c.order != 1 && c.order != 2 && (c.order != 3 || L.kind != JACC_LOOP_HEAT3D)) return 1;
            if (c.march != 1 && c.march != 2) return 1;
            if (c.rows != 1 && (L.kind != JACC_LOOP_HEAT3D || c.persistent)) return 1;
            if (c.rows != 1 && c.rows != 2 && c.rows != 4 && c.rows != 8) return 1;
            if (c.rows != 1 && c.bx * c.by > 256) return 1;  // multi-row waves: workgroups of at most 256
            return 0;
        case JACC_LOOP_GEMM:
            // k-slab depth and workgroup size; other fields are ignored
            return ((c.tile == 16 || c.tile == 32) && (c.bx == 256 || c.bx == 512)) ? 0 : 1;
        case JACC_LOOP_SPMV_CSR:
            // order 4: column-banded, by = bands per XCD, tile = lanes per
            // row and band (1 to 16)
            if (c.order == 4)
                return ((c.tile == 1 || c.tile == 2 || c.tile == 4 || c.tile == 8 || c.tile == 16) &&
                        (c.by == 1 || c.by == 2 || c.by == 4 || c.by == 8) &&
                        (c.rows == 1 || (c.tile == 1 && (c.rows == 2 || c.rows == 4))))
                           ? 0
                           : 1;
            if (c.tile != 4 && c.tile != 8 && c.tile != 16) return 1;
            return (c.order == 1 || c.order == 2) ? 0 : 1;
        case JACC_LOOP_SUM:
        case JACC_LOOP_SCATTER_SQ:
        case JACC_LOOP_PRED_CHAIN:
            return 0;  // fixed internal configurations; fields are ignored
        default:
            return 1;
    }
}

int64_t reduction_workgroups(const Launch &L) {
    switch (L.kind) {
        case JACC_LOOP_HEAT3D: return heat3d_workgroups(L);
        case JACC_LOOP_SUM: return sum_workgroups(L);
        default: return 0;
    }
}

hipError_t launch_loop(const Launch &L, hipStream_t s) {
    switch (L.kind) {
        case JACC_LOOP_JACOBI2D: return launch_jacobi2d(L, s);
        case JACC_LOOP_HEAT3D: {
            hipError_t e = launch_heat3d(L, s);
            if (e != hipSuccess || !L.wg_partials) return e;
            return launch_finalise(L.wg_partials, heat3d_workgroups(L), L.part_out, s);
        }
        case JACC_LOOP_SUM: return launch_sum(L, s);
        case JACC_LOOP_GEMM: return launch_gemm(L, s);
        case JACC_LOOP_SPMV_CSR: return launch_spmv(L, s);
        case JACC_LOOP_SCATTER_SQ: return launch_scatter(L, s);
        case JACC_LOOP_PRED_CHAIN: return launch_chain(L, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace jk
