"""MI355X (gfx950) label propagation: the nu-LPA label sweep (arXiv 2411.11468)
as hand-written HIP kernels behind a C ABI (include/lpa.h, liblpa.so).

Build the library with ``python -m paper_2411_11468_amd.build``.
"""
from .lpa import (LAUNCH_EAGER, LAUNCH_GRAPH, MODE_ASYNC, MODE_DETERMINISTIC,
                  BatchResult, LpaBatch, LpaError, LpaGraph, Predictor, RunResult, default_options,
                  default_tuning, load_library, lpa_create, lpa_create_batched, lpa_destroy,
                  lpa_graph_classes, lpa_modularity, lpa_run, lpa_run_batched)

__all__ = ["LAUNCH_EAGER", "LAUNCH_GRAPH", "MODE_ASYNC", "MODE_DETERMINISTIC", "BatchResult",
           "LpaBatch", "LpaError", "LpaGraph", "Predictor", "RunResult", "default_options",
           "default_tuning", "load_library", "lpa_create", "lpa_create_batched",
           "lpa_destroy", "lpa_graph_classes", "lpa_modularity", "lpa_run",
           "lpa_run_batched"]
