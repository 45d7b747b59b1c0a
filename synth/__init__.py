from .grid_ls import GridProblem, general_ls, grid_ls, grid_square, config_problem, batch_problem, batch_sides, default_depth, CONFIGS  # noqa: F401
from .inverse_poisson import inverse_poisson  # noqa: F401
