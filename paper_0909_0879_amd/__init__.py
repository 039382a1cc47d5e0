"""MI355X-native direct N-body hot path: O(N^2) softened acceleration and
jerk (eq. (1) of the paper), Hermite-4 block time steps, ensembles of
independent clusters.  The compute lives in libnbody.so (HIP, gfx950,
C ABI in include/nbody.h); `binding` marshals torch tensors into it and
`ics` draws seeded synthetic initial conditions."""
__all__ = ["binding", "ics"]
