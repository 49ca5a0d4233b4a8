"""Launch shapes (tx, ty, cz) of the fused step for the standard workloads,
picked by ``lbm_autotune`` on an MI355X.  Any shape is correct; these are
the measured fastest."""

STEP_TILES = {
    # (workload, storage) -> (tx, ty, cz)
    ("droplet_32", "f64"): (32, 8, 8),
    ("laplace_128", "f64"): (64, 4, 16),
    ("laplace_128", "f32"): (64, 4, 16),
    ("two_droplets_256", "f64"): (128, 4, 64),
    ("two_droplets_256", "f32"): (64, 4, 32),
    ("two_droplets_256", "f16s"): (64, 4, 32),
    ("sessile_384x384x192", "f32"): (64, 4, 32),
}


def tile_for(workload: str, storage: str):
    return STEP_TILES.get((workload, storage))
