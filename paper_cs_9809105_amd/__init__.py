"""Hyper-systolic matrix products on AMD MI355X (gfx950)."""
