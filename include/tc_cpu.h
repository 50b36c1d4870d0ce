/* Multicore CPU census (context baseline, not part of the GPU path).
 *
 * The thesis's host variant (section v0.7, "local census array per thread",
 * with the task queues of figure "Canonical Dyad (uniform distr.)" and the
 * pre-computed dyad type of v0.4): canonical dyads split into runs of rows of
 * about equal sum of |N(u)| + |N(v)|, handed out to the threads, one local
 * census per thread, summed after the join.  Within a dyad the one-sided third
 * vertices come from per-row prefix counts and the shared ones from one merge
 * of the two sorted rows.  Counts are exact and equal to tc_census's.
 */
#ifndef TC_CPU_H
#define TC_CPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Census of the digraph with m arcs src[i] -> dst[i] (host int32 ids in
 * [0, n); loops dropped, repeated arcs merged).  threads <= 0 uses every
 * hardware thread.  counts[16] receives the class counts in the thesis's order;
 * *census_seconds (may be null) the wall time of the census after the
 * adjacency is built.  The caller owns every buffer; nothing is retained.
 * Returns 0, or -1 on a null pointer, a negative size or an id out of range
 * (outputs untouched). */
int tc_cpu_census(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t threads,
                  uint64_t counts[16], double* census_seconds);

#ifdef __cplusplus
}
#endif

#endif
