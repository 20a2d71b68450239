"""Plain FP64 CPU oracle for the coupled LBM / momentum-exchange / rigid-fiber
method.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
CPU-baseline leg of the benchmark may load it; the GPU library never does."""
