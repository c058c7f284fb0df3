"""MI355X-native hot path of YAND-MVSK (Yau's affine-normal descent for
unrestricted mean-variance-skewness-kurtosis portfolios).

All computation runs in libyand.so (hand-written HIP kernels for gfx950);
this package only marshals arguments.  Importing it does not touch the GPU;
the first call loads the library and fails loudly if it or the GPU is absent.
"""

from .binding import (  # noqa: F401
    Context,
    Mlp,
    SolveInfo,
    YandError,
    batch_solve,
    default_mlp_opts,
    default_opts,
    from_reduced,
    is_certified_convex,
    load,
    project_simplex,
    reduced_coords,
    solve_R,
    warmstart_features,
    warmstart_predict,
    warmstart_train,
    LIB_PATH,
)
