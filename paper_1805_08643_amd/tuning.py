"""Launch shapes (tx, ty, cz) and step kernels for the standard workloads,
measured fastest on an MI355X (``lbm_autotune`` and sweeps).  Any shape and
either kernel give the same populations; these are the fastest found."""

STEP_TILES = {
    # (workload, storage, mode) -> (tx, ty, cz); mode "fused": one node per
    # thread, "pairs" / "quads": two / four x-adjacent nodes per thread, "split":
    # 8-byte groups (four F16S or two FP32 nodes) with pulling and colliding
    # waves (tx counts nodes)
    ("droplet_32", "f64", "fused"): (32, 2, 4),
    ("laplace_128", "f64", "fused"): (128, 4, 16),
    ("laplace_128", "f32", "fused"): (64, 4, 16),
    ("laplace_128", "f32", "pairs"): (64, 8, 8),
    ("laplace_128", "f32", "split"): (128, 4, 16),
    ("laplace_128", "f16s", "fused"): (64, 8, 16),
    ("laplace_128", "f16s", "pairs"): (64, 8, 8),
    ("laplace_128", "f16s", "split"): (64, 16, 8),
    ("two_droplets_256", "f64", "fused"): (128, 4, 128),
    ("two_droplets_256", "f32", "fused"): (64, 4, 128),
    ("two_droplets_256", "f32", "pairs"): (128, 8, 64),
    ("two_droplets_256", "f32", "split"): (128, 4, 128),
    ("two_droplets_256", "f16s", "fused"): (64, 4, 32),
    ("two_droplets_256", "f16s", "pairs"): (128, 8, 64),
    ("two_droplets_256", "f16s", "quads"): (128, 16, 32),
    ("two_droplets_256", "f16s", "split"): (128, 8, 64),
    ("two_droplets_256", "f16n", "split"): (128, 8, 64),
    ("sessile_384x384x192", "f32", "fused"): (64, 4, 32),
    ("sessile_384x384x192", "f32", "pairs"): (128, 8, 16),
    ("sessile_384x384x192", "f32", "split"): (128, 4, 48),
    ("sessile_384x384x192", "f16n", "split"): (128, 8, 32),
}

# Faster step kernel per (workload, storage); absent: "fused".
STEP_MODES = {
    ("laplace_128", "f32"): "split",
    ("laplace_128", "f16s"): "split",
    ("two_droplets_256", "f32"): "split",
    ("two_droplets_256", "f16s"): "split",
    ("sessile_384x384x192", "f32"): "split",
}


def mode_for(workload: str, storage: str) -> str:
    if storage == "f16n":  # the split step is F16N's only kernel
        return "split"
    return STEP_MODES.get((workload, storage), "fused")


def tile_for(workload: str, storage: str, mode: str = "fused"):
    return STEP_TILES.get((workload, storage, mode))
