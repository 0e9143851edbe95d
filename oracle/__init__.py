"""CPU oracle for the dense OMM path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may import
this package. The HIP library and its binding never import it and share no code with it.
"""
