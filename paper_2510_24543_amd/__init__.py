"""MI355X-native preconditioned nonlinear CG ground-state solver (package root)."""
