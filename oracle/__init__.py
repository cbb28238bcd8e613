"""CPU oracle of the multiresolution block-octree method (plain FP64).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product path (the HIP
library and its Python binding) never imports, links or executes it.
"""
