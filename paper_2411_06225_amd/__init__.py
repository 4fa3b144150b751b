"""RandNet-Parareal on AMD MI355X (placeholder during bring-up)."""
