"""Batch-dynamic rooted spanning forest (D-RSF) on AMD MI355X.

The compute path is libdrsf.so (HIP, gfx950), built from csrc/ and declared
in include/drsf.h; this package is its ctypes binding.
"""
from .drsf import (DRSF_DELETE, DRSF_INSERT, DrsfError, Forest, MultiForest, Server, drsf_apply,
                   drsf_apply_async, drsf_copy_out, drsf_create, drsf_default_opts,
                   drsf_destroy, drsf_export_edges, drsf_multi_apply, drsf_multi_apply_async,
                   drsf_multi_create, drsf_multi_num_edges, drsf_multi_wait, drsf_num_edges,
                   drsf_num_graphs, drsf_phase_times, drsf_set_tuning, drsf_snapshot_free,
                   drsf_snapshot_restore, drsf_snapshot_take, drsf_version, drsf_wait, load)

__all__ = ["DRSF_DELETE", "DRSF_INSERT", "DrsfError", "Forest", "MultiForest", "Server", "drsf_apply",
           "drsf_apply_async", "drsf_copy_out", "drsf_create", "drsf_default_opts",
           "drsf_destroy", "drsf_export_edges", "drsf_multi_apply", "drsf_multi_apply_async",
           "drsf_multi_create", "drsf_multi_num_edges", "drsf_multi_wait", "drsf_num_edges",
           "drsf_num_graphs", "drsf_phase_times", "drsf_set_tuning", "drsf_snapshot_free",
           "drsf_snapshot_restore", "drsf_snapshot_take", "drsf_version", "drsf_wait", "load"]
