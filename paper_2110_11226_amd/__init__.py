"""MI355X (gfx950) GP population evaluation: the data-parallel hot path of
stack-based generational genetic programming (arXiv 2110.11226).

The work happens in ``libgp.so`` (HIP kernels + host C++ behind the C ABI of
``include/gp.h``); this package binds it.  Importing it without the built
library raises ImportError.
"""
from ._binding import (  # noqa: F401
    DeviceDataset, DevicePopulation, GPError, HostPopulation, build_population, evaluate,
    fitness, fitness_backward, fitness_noalloc, larger_is_better, metric_id, shutdown, tournament,
    validate_population, version, get_launch_config, set_launch_config, set_spearman_workset,
    profile_enable, profile_read, autotune, autotune_save, autotune_load, autotune_clear, Generation,
    plan_generation, mutate, GENOPS, plan_generation_device, mutate_device, DeviceOffspring, FUNCS_ALL, Evolution,
    FUNCS_DEFAULT, MAX_STACK, METRICS, LIB_PATH, register_function, function_defined, OP_USER1, OP_USER2,
)
from .autograd import GPFitness, refine_constants  # noqa: F401,E402
from .loop import (run_generations, RunResult, GenerationLog, save_checkpoint,  # noqa: F401,E402
                   load_checkpoint)
