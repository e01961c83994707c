"""Seeded synthetic inputs shared by the oracle tests and the HIP path:
mechanism draws, primitive initial fields and the named workloads.  Holds
none of the method's arithmetic."""
