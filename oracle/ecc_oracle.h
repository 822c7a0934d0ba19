/*
 * C entry points of the all-levels oracle (O2), TEST INFRASTRUCTURE ONLY:
 * only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg load
 * the library built from ec_oracle_o2.c.  It shares no header, code or
 * table with the HIP library; the two structs below are laid out like the
 * library's field and curves descriptors, so that the same request can be
 * handed to both, but they are declared here on their own.
 *
 * What is computed: the curves of the Methodology section, Eq. (1) over the
 * filtration of Eq. (2) (or its superlevel mirror), from the level at which
 * every cubical cell enters, all levels at once.
 */
#ifndef ECC_ORACLE_H
#define ECC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A field and its filtration, HOST pointers.
 *   ndim 2 or 3; dtype 1 = uint8, 2 = uint16, 3 = float32;
 *   shape {h, w} or {d, h, w}, C order, each >= 1;
 *   n_levels L >= 1;
 *   connectivity 2D 8 or 4, 3D 26 or 6, 0 = 8 / 26;
 *   thresholds NULL (integer levels) or L float32 values, non-decreasing
 *   (sublevel: active when value <= t_l) or non-increasing (superlevel:
 *   active when value >= t_l; integer levels t_l = L - 1 - l);
 *   filtration 0 = sublevel, 1 = superlevel. */
typedef struct {
    int32_t ndim;
    int32_t dtype;
    int64_t shape[3];
    const void *data;
    int32_t n_levels;
    int32_t connectivity;
    const float *thresholds;
    int32_t filtration;
} ecc_oracle_field;

/* HOST int64 arrays of length L, NULL = not wanted (at least one given);
 * volume must be NULL in 2D.  3D: perimeter = crease measure, area = surface. */
typedef struct {
    int64_t *ec;
    int64_t *perimeter;
    int64_t *area;
    int64_t *volume;
} ecc_oracle_curves;

/* The curves of `field` into `curves` with up to n_threads OpenMP threads.
 * Returns 0 on success, 1 when an argument breaks a rule above (nothing is
 * written then), 3 when host memory runs out. */
int ecc_oracle_compute(const ecc_oracle_field *field, const ecc_oracle_curves *curves, int32_t n_threads);

/* The same with the arguments spelled out (the form the Python helpers call). */
int ecc_oracle_o2(int ndim, const int64_t *shape, int dtype, const void *data, int32_t n_levels,
                  const float *thresholds, int32_t connectivity, int32_t superlevel, int64_t *ec,
                  int64_t *perimeter, int64_t *area, int64_t *volume, int n_threads);

#ifdef __cplusplus
}
#endif

#endif
