"""MI355X-native native hybrid queries (NHQ, arXiv 2203.13601).

The product is ``libnhq.so`` (HIP kernels for gfx950 behind the C ABI of
``include/nhq.h``); this package is its thin Python binding.  Importing it
does not load the library; the first call does, and raises if the library
has not been built.
"""
from ._binding import (BuildParams, Index, NHQError, SearchParams, lib,  # noqa: F401
                       nhq_bruteforce_hybrid_knn, nhq_build_index, nhq_hybrid_search,
                       nhq_index_build_graph, nhq_index_create, nhq_index_device_error,
                       nhq_index_get_entry, nhq_index_get_graph, nhq_index_get_storage, nhq_index_info,
                       nhq_index_set_graph, nhq_search_seeded, nhq_seed_rank, nhq_seed_rank_workspace_size,
                       DEVERR_BADID, DEVERR_HOPCAP, STORAGE,
                       MLP_PARAMS, TraceBuffers, nhq_mlp_eval, nhq_mlp_grad, nhq_mlp_load, nhq_mlp_train,
                       nhq_trace_samples, Server, ServerParams, nhq_server_create, SERVE_RAW, nhq_gather_probe,
                       nhq_nndescent_lists, nhq_index_build_report, WEIGHTS, BUILDERS,
                       nhq_index_insert, nhq_index_save, nhq_index_load,
                       nhq_hybrid_search_noalloc, NOALLOC_SCRATCH_BYTES,
                       nhq_index_entry_blocks, nhq_query_order, nhq_seed_order)
