"""MI355X subset digital image correlation: brute-force and particle swarm
ZNCC integer searches, IC-GN and Newton-Raphson sub-pixel refinement and the
ZNSSD adjoint, as HIP kernels behind the C ABI in include/dic.h (libdic.so),
with a thin ctypes binding."""
from .dic import (FLAG_BICUBIC_LUT, FLAG_CACHE_REF_PREP, FLAG_DETERMINISTIC_BWD,  # noqa: F401
                  FLAG_INTERP_BILINEAR, FLAG_INTERP_BSPLINE,
                  FLAG_REFINE_NR, FLAG_USE_GRAPH,
                  FP32_BATCHED, FP64_PLAIN, POI_NAN_INPUT, POI_NO_VALID_CANDIDATE,
                  PSO_GENERATIONS, PSO_PARTICLES,
                  POI_NOT_CONVERGED, POI_OK, POI_OUT_OF_BOUNDS, POI_SINGULAR_HESSIAN,
                  POI_ZERO_VARIANCE, ZNSSD, DicError, PairSpec, Plan, batch_layout,
                  LatestFrame, LiveCorrelator, correlate, correlate_batch, correlate_sequence,
                  load_library, poi_grid, SequenceCheckpoint, STATUS_NAMES,
                  single_pair_plan, status_histogram)
