/*
 * CPU oracle for the XCSR multigraph transpose -- test infrastructure only.
 * Declarations for oracle.c; this header belongs to the oracle alone.
 */
#ifndef MGO_ORACLE_H
#define MGO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { MGO_OK = 0, MGO_EINVAL = -1, MGO_ERANGE = -2, MGO_ENOMEM = -3, MGO_EUNSUPPORTED = -5 };

/* ow = offset width in bytes (4 or 8) of row_ptr / payload_off / outputs. */
int mgo_validate(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                 const int32_t* col, const void* payload_off, int32_t R, const int64_t* bounds);

int mgo_transpose(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                  const int32_t* col, const void* payload_off, const uint8_t* payload,
                  void* t_row_ptr, int32_t* t_col, void* t_payload_off, uint8_t* t_payload,
                  uint32_t* perm);

int mgo_partition_counts(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                         const int32_t* col, const void* payload_off, int32_t R,
                         const int64_t* bounds, int64_t* xfer_cells, int64_t* xfer_bytes,
                         int64_t* part_cell_off, int64_t* part_byte_off, int64_t* sdispls,
                         int64_t* rdispls);

int mgo_transpose_columns(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                          const int32_t* col, const void* payload_off, const uint8_t* payload,
                          int64_t c_lo, int64_t c_hi, int64_t* t_row_ptr_slice,
                          int32_t* t_col_slice, int64_t* t_payload_off_slice,
                          uint8_t* t_payload_slice, uint32_t* perm_slice, int64_t* cells_out,
                          int64_t* bytes_out);

#ifdef __cplusplus
}
#endif
#endif
