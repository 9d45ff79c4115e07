"""MI355X-native thermal lattice Boltzmann solver with characteristic boundary conditions.

Hot path (HIP, gfx950) behind the C-ABI library ``liblbm_hip.so`` (declared in include/lbm.h);
``lbm`` is the thin Python binding (argument marshalling only) and ``workloads`` builds the seeded
synthetic initial fields.
"""
__all__ = ["lbm", "workloads"]
