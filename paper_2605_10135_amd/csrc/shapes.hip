// shapes.hip -- one slice of the distance-kernel shape table: the kernels of
// one precision (SG_SHAPE_PREC), one selection width (SG_SHAPE_KSEL), single-
// shard or persistent batched (SG_SHAPE_BATCHED).  The build compiles this
// file once per slice, in parallel, and links every slice into the library.
#include "batch_impl.hpp"
#include "shapes.hpp"

#if !defined(SG_SHAPE_PREC) || !defined(SG_SHAPE_KSEL) || !defined(SG_SHAPE_BATCHED)
#error "shapes.hip is compiled once per slice: define SG_SHAPE_PREC, SG_SHAPE_KSEL and SG_SHAPE_BATCHED"
#endif

#if SG_SHAPE_BATCHED
template bool sg::knn::for_shapes_p<SG_SHAPE_PREC, sg::batch::BatchedMaker<SG_SHAPE_KSEL>>(
    int, sg::batch::BatchedMaker<SG_SHAPE_KSEL>&);
#else
template bool sg::knn::for_shapes_p<SG_SHAPE_PREC, sg::knn::ResidentMaker<SG_SHAPE_KSEL>>(
    int, sg::knn::ResidentMaker<SG_SHAPE_KSEL>&);
#endif
