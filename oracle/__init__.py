"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never imports,
links or calls it.  See ``oracle.c`` for what is computed and which passage
of the paper each part follows.
"""
from .pyoracle import (  # noqa: F401
    build,
    use_library,
    compile_source,
    source_text,
    lib_path,
    solve_grid,
    solve_points,
    density,
    field_A,
    field_E,
    field_table,
    field_table_y,
    field_Ay,
    field_Ey,
    composition,
    boundary_A,
    snapshot_points,
    snapshot_grid,
    state_at,
    step_matrix_xy,
    times,
    step_matrix,
    spinors,
    final_state,
    grid_p,
)
