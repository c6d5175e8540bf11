// The records-only partition pass (the last pass of a schedule of two or
// more) built with 512-thread workgroups and 4,096-cell LDS sub-chunks. Each
// sub-chunk then leaves about 16 cells per digit instead of 8, so the
// (column, size) and 16-byte (row, index, payload offset) records are written
// in runs twice as long. The other stages keep 256 threads and 2,048 cells:
// the first pass and the finish hold payload bytes or byte prefixes in LDS,
// which at 4,096 cells would leave one workgroup per CU. This form also takes
// up to 9 digit bits (fan-out 512), so a single large matrix reaches finish
// buckets of about 4,096 cells in two passes.
#define MGT_WIDE 1
#define MGT_GEO_NS geo512
#define MGT_GEO_BLOCK ::mgt::kWideBlock
#define MGT_GEO_SUB ::mgt::kWideSub
#define MGT_GEO_FANBITS ::mgt::kMaxLastPassBits
#include "kernels.hip"
