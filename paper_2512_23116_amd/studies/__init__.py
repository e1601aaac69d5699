"""Studies built on the hot path: the paper's regime diagnostic run and the
reduced-precision comparison.  Each is a module with a ``main()``."""
