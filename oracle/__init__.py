"""Plain FP64 CPU oracle of the BSSN right-hand side, RK4 step and
constraints.  Test infrastructure only: the product path never imports it."""
