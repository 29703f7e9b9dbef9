"""MI355X-native phase-insensitive quantum detector tomography (arXiv 2404.02844).

The solver lives in the HIP library ``libpdt.so`` (C ABI in ``include/pdt.h``);
``_pdt`` is its ctypes binding and ``synth`` generates seeded synthetic inputs.
"""
from . import _pdt  # noqa: F401
from ._pdt import (BatchProblem, PDT_FP32, PDT_FP64, PDT_INIT_LEARNED, PDT_MIXED, Model, pdt_warmstart_features, PDT_INIT_UNIFORM, PDT_INIT_USER, PDT_TAIL_LUMP,  # noqa: F401
                   PDT_TAIL_TRUNCATE, PdtError, Problem, pdt_destroy_problem, pdt_kkt, pdt_last_error,
                   pdt_make_problem, pdt_objective, pdt_problem_bands, pdt_problem_scaling, pdt_project_simplex, pdt_solve,
                   PDT_STEP_UNIFORM, PDT_STEP_DIAG, pdt_hessian_apply, pdt_newton_direction, pdt_newton_solve,
                   pdt_smooth_rows)
