"""MI355X (gfx950) label propagation: the nu-LPA label sweep (arXiv 2411.11468)
as hand-written HIP kernels behind a C ABI (include/lpa.h, liblpa.so).

Build the library with ``python -m paper_2411_11468_amd.build``.
"""
from .lpa import (LpaError, LpaGraph, RunResult, default_options, default_tuning,
                  load_library, lpa_create, lpa_destroy, lpa_graph_classes,
                  lpa_modularity, lpa_run, MODE_ASYNC, MODE_DETERMINISTIC)

__all__ = ["LpaError", "LpaGraph", "RunResult", "default_options", "default_tuning",
           "load_library", "lpa_create", "lpa_destroy", "lpa_graph_classes",
           "lpa_modularity", "lpa_run", "MODE_ASYNC", "MODE_DETERMINISTIC"]
