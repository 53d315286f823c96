"""Seeded synthetic inputs (conductivity fields, flow solve, particle release).

Shared by the oracle tests and the GPU path; holds none of the tracking
arithmetic.
"""


def workload(name: str):
    """The named seeded workload: C1-C6 (workloads.configs) or C7 (workloads.quadtree)."""
    from . import configs, quadtree
    if name == "C7":
        return quadtree.c7()
    if name in configs.CONFIGS:
        return configs.CONFIGS[name]()
    raise KeyError("unknown workload " + name)
