// Adaptive choice between duplicated and partitioned execution of one loop
// nest (Sec. "Adaptive Utilization", Eq. 1-3).
//
// A loop starts in duplicate mode (one device computes the whole loop; no
// exchange).  The first observation is a warm-up and is ignored.  Every
// later duplicate-mode observation adds time/WriteSize to the running mean
// eff_dup (seconds per byte written) and is tested against Eq. 1,
//     t_kernel > t_kernel / n + WriteSize / peak_p2p;
// after five executions that satisfy it the loop switches to partitioned
// mode.  In partitioned mode each observation (kernel time of a partition,
// exchange time) is tested against Eq. 2, t_k + t_c > n * t_k, and Eq. 3,
// t_k + t_c > eff_dup * WriteSize; once either has held five times and the
// mean, over every partitioned execution since the switch, of the left side
// minus the smaller right side is above zero, the loop returns to duplicate
// mode for good.  Executions that beat both bounds contribute negative
// differences, so a loop that is mostly faster partitioned stays partitioned
// through occasional violations.
//
// Host-only bookkeeping; it launches nothing and allocates one small record.
#include <cmath>
#include <new>

#include "jacc.h"

struct jacc_adapt {
    int n = 1;
    double peak = 0.0;
    int mode = JACC_ADAPT_DUPLICATE;
    bool warmed = false;
    long long n_dup = 0, n_eq1 = 0, c2 = 0, c3 = 0, n_viol = 0, n_part = 0;
    double sum_ratio = 0.0, sum_diff = 0.0;
};

extern "C" {

int jacc_adapt_create(jacc_adapt **out, int n_parts, double peak_bytes_per_s) {
    if (!out) return JACC_ERR_INVALID;
    *out = nullptr;
    if (n_parts < 1 || !(peak_bytes_per_s > 0.0) || !std::isfinite(peak_bytes_per_s)) return JACC_ERR_INVALID;
    jacc_adapt *a = new (std::nothrow) jacc_adapt;
    if (!a) return JACC_ERR_ALLOC;
    a->n = n_parts;
    a->peak = peak_bytes_per_s;
    *out = a;
    return JACC_OK;
}

int jacc_adapt_destroy(jacc_adapt *a) {
    delete a;
    return JACC_OK;
}

int jacc_adapt_observe(jacc_adapt *a, double time_kernel_s, double time_comm_s, double write_bytes, int *mode) {
    if (!a || !(time_kernel_s >= 0.0) || !(time_comm_s >= 0.0) || !(write_bytes > 0.0) ||
        !std::isfinite(time_kernel_s) || !std::isfinite(time_comm_s) || !std::isfinite(write_bytes))
        return JACC_ERR_INVALID;
    if (a->mode == JACC_ADAPT_PARTITION) {
        const double eff_dup = a->sum_ratio / (double)a->n_dup;
        const double left = time_kernel_s + time_comm_s;
        const double r2 = time_kernel_s * a->n;       // Eq. 2
        const double r3 = eff_dup * write_bytes;      // Eq. 3
        const bool v2 = left > r2, v3 = left > r3;
        if (v2) ++a->c2;
        if (v3) ++a->c3;
        if (v2 || v3) ++a->n_viol;
        ++a->n_part;
        a->sum_diff += left - (r2 < r3 ? r2 : r3);
        if ((a->c2 >= 5 || a->c3 >= 5) && a->sum_diff / (double)a->n_part > 0.0) a->mode = JACC_ADAPT_DUPLICATE_FINAL;
    } else if (!a->warmed) {
        a->warmed = true;  // the warm-up run is not profiled
    } else if (a->mode == JACC_ADAPT_DUPLICATE) {
        ++a->n_dup;
        a->sum_ratio += time_kernel_s / write_bytes;
        if (time_kernel_s > time_kernel_s / a->n + write_bytes / a->peak) ++a->n_eq1;  // Eq. 1
        if (a->n_eq1 >= 5) a->mode = JACC_ADAPT_PARTITION;
    }
    if (mode) *mode = a->mode;
    return JACC_OK;
}

int jacc_adapt_state(const jacc_adapt *a, int *mode, double *eff_dup, long long *counts) {
    if (!a) return JACC_ERR_INVALID;
    if (mode) *mode = a->mode;
    if (eff_dup) *eff_dup = a->n_dup ? a->sum_ratio / (double)a->n_dup : 0.0;
    if (counts) {
        counts[0] = a->n_dup;
        counts[1] = a->n_eq1;
        counts[2] = a->c2;
        counts[3] = a->c3;
        counts[4] = a->n_viol;
    }
    return JACC_OK;
}

int jacc_adapt_mean_diff(const jacc_adapt *a, double *mean_diff, long long *n_partitioned) {
    if (!a) return JACC_ERR_INVALID;
    if (mean_diff) *mean_diff = a->n_part ? a->sum_diff / (double)a->n_part : 0.0;
    if (n_partitioned) *n_partitioned = a->n_part;
    return JACC_OK;
}

}  // extern "C"
