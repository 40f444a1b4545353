"""CPU FP64 oracle for the EA/IP-ADC(n) hot path.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import anything in this package.  It shares no code with
the HIP library.
"""
