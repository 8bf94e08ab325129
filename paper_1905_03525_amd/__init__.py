"""MI355X (gfx950) linear-work R-MAT edge sampler (Huebschle-Schneider & Sanders,
arXiv 1905.03525).  The HIP library librmat.so implements the C ABI of
include/rmat.h and include/rmat_serve.h; this package binds it under the same
names."""
from .rmat import (RMAT_EDEVICE, RMAT_EINVAL, RMAT_ENOMEM, RMAT_ERANGE, RMAT_FIXED, RMAT_OK,  # noqa: F401
                   RMAT_REQ_DIGEST, RMAT_REQ_DISCARD, RMAT_SCRAMBLE, RMAT_UNDIRECTED, RMAT_VARIABLE, Batch, RmatError, Server, Table,
                   generate_edges, generate_partition, id_dtype, load, make_instances, make_request, rmat_batch_autotune,
                   rmat_batch_check, rmat_batch_create, rmat_batch_enqueue, rmat_batch_free, rmat_batch_get_info,
                   rmat_batch_launch_graph, rmat_batch_table_export, rmat_batch_table_info, rmat_build_table,
                   rmat_build_table_async,
                   rmat_kron_build_table, rmat_build_perturbed_table, rmat_table_export_member,
                   rmat_free_table, rmat_generate, rmat_generate_async, rmat_generate_ex_async, rmat_generate_partition, rmat_generate_partition_async, rmat_generate_reduce_async, rmat_generate_reduce_noalloc_async,
                   rmat_generate_degrees_async, rmat_degree_distribution_async,
                   rmat_last_error, rmat_partition_counts, rmat_server_clock, rmat_server_create, rmat_server_drain, rmat_server_free,
                   rmat_server_get_stats, rmat_server_poll, rmat_server_release, rmat_server_run_trace,
                   rmat_server_step, rmat_server_submit, rmat_table_export, rmat_table_info, to_numpy_ids)
