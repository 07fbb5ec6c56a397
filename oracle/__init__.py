"""FP64 CPU oracle of the PIC-MCC diode: test infrastructure only (tests, smoke check,
CPU-baseline leg of the benchmark).  The product path never imports it."""
