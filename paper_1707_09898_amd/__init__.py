"""MI355X-native gradient engine for FD topology optimization of permanent magnets."""
