"""Test oracle for the vdW-DF nonlocal-correlation path (test infrastructure only).

Plain FP64 CPU reference written from the paper's definitions; shares no
code with the HIP library.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import it.
"""
