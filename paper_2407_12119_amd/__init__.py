"""MI355X-native batched GNN track finding for the LHCb VELO (arXiv 2407.12119).

Submodules:
  velo   -- Python binding of libvelognn.so (the HIP path, include/velognn.h)
  synth  -- seeded synthetic events and parameters (the shared input generator)
  metrics-- track-finding metrics of the paper's Table 1 (host-side evaluation)
  build  -- hipcc build of libvelognn.so
The library is loaded lazily by `velo.lib()`.
"""
