"""MI355X (gfx950) linear-work R-MAT edge sampler (Huebschle-Schneider & Sanders,
arXiv 1905.03525).  The HIP library librmat.so implements the C ABI of
include/rmat.h; this package binds it under the same names."""
from .rmat import (RMAT_EDEVICE, RMAT_EINVAL, RMAT_ENOMEM, RMAT_ERANGE, RMAT_FIXED, RMAT_OK, RMAT_VARIABLE,
                   Batch, RmatError, Table, generate_edges, id_dtype, load, make_instances, rmat_batch_autotune,
                   rmat_batch_check, rmat_batch_create, rmat_batch_enqueue, rmat_batch_free,
                   rmat_batch_get_info, rmat_batch_launch_graph, rmat_batch_table_export, rmat_batch_table_info, rmat_build_table,
                   rmat_free_table, rmat_generate, rmat_generate_async, rmat_generate_reduce_async,
                   rmat_last_error, rmat_table_export, rmat_table_info, to_numpy_ids)
